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
// Pipelining: sweep s+1 may run step k once sweep s has completed step k+1
// and has stored the first entry (beta) of the pivot column of its step k+2.
// Step k+2 of sweep s touches exactly one entry that step k of sweep s+1
// also touches: that beta, in the last row of the block below the diagonal
// block.  The pivot column of step k+2 is column 0 of the block below the
// diagonal block of step k+1, so step k+1 forms the next reflector itself
// and stores (beta, 0, ..., 0) in place of that column together with its own
// updates.  Every other pair of steps that touches a common entry is ordered
// by the completion of step k+1.  The per-sweep counter progress[s] holds
// 2*(steps completed) + 1 (the next step's beta is then in memory too), and
// 2*nsteps + 1 when the sweep is done; a waiting step needs
// min(2k + 5, 2 nsteps(s) + 1).  Every wait is bounded.
//
// Sweeps are handed out in ascending order by an atomic ticket: a workgroup
// takes the next sweep when it has finished its previous one.  A sweep only
// waits for the sweep before it, which a running workgroup took earlier, so
// the chain always moves whether or not every workgroup of the launch is
// resident at once (no cooperative launch is needed, and the kernel can share
// the device with other streams' work).
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
// sweep writes it between the two steps except for the beta entry, which is
// in place before the step's wait ends.  It therefore stays in LDS (two
// buffers, alternating) and the next reflector is computed from it at the
// end of the step; only the new below block and the last row of the
// diagonal block are loaded after the wait of the next step.
//
// Thread (tx, ty) = (tid % 64, tid / 64) owns row tx and columns ty + 4q
// (q = 0..15) of the 64 x 64 blocks, so every global access of a wavefront is
// one contiguous run of a band column and no index needs a division.
//
// One launch chases one band (lanes = null: ticket t is sweep t of `one`) or
// a batch of bands: the problems are dealt to M lanes, each lane a list of
// problems whose sweeps follow each other, and ticket t is position t / M of
// lane t % M.  A sweep waits only for the previous sweep of its own problem,
// whose ticket is smaller, so the same progress argument holds, and M
// problems advance side by side.
__global__ __launch_bounds__(256) void k_bulge_chase(skew::ChaseProb one, const skew::ChaseProb *__restrict__ probs,
                                                     const int *__restrict__ lanes, int M, int maxlen,
                                                     unsigned *ticket)
{
    __shared__ double vv[2][64], wv[64], dots[64], y2[64];
    __shared__ double pw[4][64], py[4][64], pd[4][64];
    __shared__ double dia[64 * CH_LD];
    __shared__ double junk[64];
    __shared__ double bw[2][64 * CH_LD];
    __shared__ double tau_s[2];
    __shared__ int abort_flag, s_next, p_next;
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    if (tid == 0) abort_flag = 0;
    __syncthreads();

    // Householder reflector of x (L entries, lane i of wavefront 0 holds x_i)
    // into buffer p (v with v_0 = 1, and tau); returns beta in every lane.
    auto reflector = [&](double xi, int L, int p) -> double {
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
        vv[p][tid] = (tid == 0) ? 1.0 : ((tid < L) ? xi * scale : 0.0);
        if (tid == 0) tau_s[p] = t;
        return beta;
    };

    for (;;) {
        __syncthreads();                          // every thread has read the previous ticket
        if (tid == 0) {
            const int t = (int)atomicAdd(ticket, 1u);
            if (!lanes) {
                s_next = t;
                p_next = (t < one.n - 2) ? -1 : -2;
            } else if (t >= M * maxlen) {
                p_next = -2;                      // every lane is exhausted
            } else {
                // lanes: [M + 1] item ranges, then items (problem, first position)
                const int l = t % M, pos = t / M;
                const int i0 = lanes[l], i1 = lanes[l + 1];
                const int *it = lanes + M + 1;
                int p = -3, s0 = 0;
                for (int i = i0; i < i1; ++i) {
                    const int q = it[2 * i], first = it[2 * i + 1];
                    if (pos >= first && pos < first + max(probs[q].n - 2, 0)) {
                        p = q;
                        s0 = first;
                    }
                }
                p_next = p;                       // -3: past the end of this lane
                s_next = pos - s0;
            }
        }
        __syncthreads();
        // the same in every lane: made explicit so that the problem's
        // parameters and addresses stay scalar
        const int pn = __builtin_amdgcn_readfirstlane(p_next);
        const int s = __builtin_amdgcn_readfirstlane(s_next);
        if (pn == -2) break;
        if (pn == -3) continue;
        const skew::ChaseProb P = (pn >= 0) ? probs[pn] : one;
        double *__restrict__ ab = P.ab;
        double *__restrict__ V2 = P.V2;
        double *__restrict__ tau2 = P.tau2;
        const int *__restrict__ goff = P.goff;
        unsigned *progress = P.progress, *err = P.err;
        const int ldab = P.ldab, n = P.n, b = P.b, nb2 = P.nb2;
        const int nst = nsteps_of(n, b, s);
        const int nprev = (s > 0) ? nsteps_of(n, b, s - 1) : 0;
        const int sig = s / nb2, col = s % nb2;
        int cur = 0;                              // buffer holding the previous below block
        int vc = 0;                               // buffer holding this step's reflector
        for (int k = 0; k < nst; ++k) {
            const int lo = s + 1 + k * b;
            const int c = (k == 0) ? s : lo - b;
            const int hi = min(lo + b - 1, n - 1);
            const int L = hi - lo + 1;
            const int bhi = min(hi + b, n - 1);
            const int L2 = bhi - hi;
            const int nlc = lo - c - 1;           // 0 for k = 0, b - 1 otherwise
            const bool more = k + 1 < nst;
            const double *lb = bw[cur];           // previous below block: rows R_k, cols R_{k-1}
            double *nb = bw[cur ^ 1];
            const double *v = vv[vc];
            // Diagonal block (strict lower part).  Every load is issued at a
            // valid band position (clamped) and scaled by 0 or 1: a test
            // around a load becomes a branch per load; the band storage holds
            // finite values everywhere.
            double vd[16], vb[16];
            auto load_dia = [&]() {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = ty + 4 * q;
                    const size_t cj = (size_t)min(lo + jl, n - 1) * ldab;
                    vd[q] = ld_coh(&ab[cj + min(max(tx - jl, 0), 2 * b)]);
                }
            };
            // full skew block in LDS from vd (zeros outside L x L); the lanes
            // with nothing to write store to junk instead of branching
            auto write_dia = [&]() {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = ty + 4 * q;
                    const double d = (tx < L && tx > jl) ? vd[q] : 0.0;
                    double *p1 = (tx >= jl) ? &dia[tx * CH_LD + jl] : &junk[tx];
                    double *p2 = (tx > jl) ? &dia[jl * CH_LD + tx] : &junk[tx];
                    *p1 = d;
                    *p2 = -d;
                }
            };
            // For k > 0 the wait of step k - 1 ensured that the previous sweep
            // completed its step k; after that only its step k + 1 writes the
            // block, in the last row (left block of that step), so all other
            // rows are loaded, and put into LDS, before the wait.  The loads
            // are issued before the poll and consumed after it.
            if (k > 0) load_dia();
            if (s > 0) {
                if (tid == 0) {
                    const unsigned need = (unsigned)min(2 * k + 5, 2 * nprev + 1);
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
                if (k > 0) write_dia();
                __syncthreads();
                if (abort_flag) return;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            } else if (k > 0) {
                write_dia();
            }
            // new below block and the last row of the diagonal block (lane j
            // of wavefront 0 holds its entry j; for k = 0 the whole block),
            // all loads issued before use
            double xr = 0.0;
            {
                double x0v = 0.0;
                if (k == 0 && tid < 64 && tid < L) x0v = ld_coh(&ab[(size_t)c * ldab + (lo + tid - c)]);
                const bool rowb = tx < L2;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = ty + 4 * q;
                    const size_t cj = (size_t)min(lo + jl, n - 1) * ldab;
                    const double xb = ld_coh(&ab[cj + min(max(hi + 1 + tx - lo - jl, 0), 2 * b)]);
                    vb[q] = xb * ((rowb && jl < L) ? 1.0 : 0.0);
                }
                if (ty == 0) {
                    const double x = ld_coh(&ab[(size_t)min(lo + tx, n - 1) * ldab + max(L - 1 - tx, 0)]);
                    xr = x * ((tx < L - 1) ? 1.0 : 0.0);
                }
                if (k == 0) {
                    load_dia();
                    write_dia();
                }
                // the first reflector of the sweep, from column s
                if (k == 0 && tid < 64) {
                    const double beta = reflector(x0v, L, vc);
                    if (tid < L) st_coh(&ab[(size_t)c * ldab + (lo + tid - c)], (tid == 0) ? beta : 0.0);
                }
                if (ty == 0 && tx < L - 1) {
                    dia[(L - 1) * CH_LD + tx] = xr;
                    dia[tx * CH_LD + L - 1] = -xr;
                }
            }
            __syncthreads();
            const double t = tau_s[vc];
            // ---- products with v: w = t A v (diagonal block), y2 = t B v
            // (below block), dots = t v^T C (left block); four partial sums
            {
                double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int jl = ty + 4 * q;
                    const double vj = v[jl];
                    a1 += dia[tx * CH_LD + jl] * vj;
                    a2 += vb[q] * vj;
                    a3 += vj * lb[jl * CH_LD + 1 + tx];
                }
                pw[ty][tx] = a1;
                py[ty][tx] = a2;
                pd[ty][tx] = a3;
            }
            __syncthreads();
            if (ty == 0) wv[tx] = t * (pw[0][tx] + pw[1][tx] + pw[2][tx] + pw[3][tx]);
            else if (ty == 1) y2[tx] = t * (py[0][tx] + py[1][tx] + py[2][tx] + py[3][tx]);
            else if (ty == 2) dots[tx] = t * (pd[0][tx] + pd[1][tx] + pd[2][tx] + pd[3][tx]);
            __syncthreads();
            // ---- updates, written back.  The new below block stays in LDS.
            // Its columns 1.. are the next step's left block, which that step
            // stores, and no other sweep reads them in between (step k-1 of
            // the next sweep reads only its column 0, step k of the next sweep
            // waits for step k+1), so only column 0 (beta, 0, ..., 0) is
            // stored.  Step k-1 of the next sweep reads the left block and
            // column 0 of the diagonal block: they are stored before the
            // publish, the rest of the diagonal block after it (the publish of
            // step k+1 waits for every earlier store; the last step of a
            // sweep stores everything before its publish).
            const double vi = v[tx], wi = wv[tx], yi = y2[tx];
            // (row L-1 of the diagonal block is held by wavefront 0, entry j
            // in lane j: xr)
            auto store_dia = [&](int q) {
                const int jl = ty + 4 * q;
                if (tx < L - 1 && tx > jl)
                    st_coh(&ab[(size_t)(lo + jl) * ldab + (tx - jl)], vd[q] + vi * wv[jl] - wi * v[jl]);
            };
            auto store_last_row = [&](bool first) {
                if (ty == 0 && tx < L - 1 && (tx == 0) == first)
                    st_coh(&ab[(size_t)(lo + tx) * ldab + (L - 1 - tx)], xr + v[L - 1] * wi - wv[L - 1] * vi);
            };
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int jl = ty + 4 * q;
                if (tx < L && jl < nlc) {
                    const int j = c + 1 + jl;
                    st_coh(&ab[(size_t)j * ldab + (lo + tx - j)], lb[tx * CH_LD + 1 + jl] - vi * dots[jl]);
                }
                nb[tx * CH_LD + jl] = vb[q] - yi * v[jl];
            }
            if (ty == 0) store_dia(0);
            store_last_row(true);
            // ---- reflector of step k + 1 from column 0 of the new below block
            // (wavefront 0 holds that column: v_0 = 1), formed while the
            // stores above are in flight; its beta and zeros are stored in
            // place of the column, so the step publishes them with its own
            // updates
            if (more && ty == 0) {
                const double beta_n = reflector(vb[0] - yi, L2, vc ^ 1);
                if (tx < L2) st_coh(&ab[(size_t)lo * ldab + (hi + 1 + tx - lo)], (tx == 0) ? beta_n : 0.0);
            }
            if (!more) {
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (q > 0 || ty > 0) store_dia(q);
                store_last_row(false);
            }
            wg_publish();
            if (tid == 0) st_relaxed(&progress[s], more ? 2u * k + 3u : 2u * nst + 1u);
            if (more) {
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (q > 0 || ty > 0) store_dia(q);
                store_last_row(false);
            }
            // ---- reflector for the back-transformation
            {
                const size_t g = (size_t)goff[sig] + k;
                if (tid < b) V2[(g * nb2 + col) * b + tid] = (tid < L) ? v[tid] : 0.0;
                if (tid == 0) tau2[g * nb2 + col] = t;
            }
            cur ^= 1;
            vc ^= 1;
        }
    }
}

// goff[sg] for sg = 0..nsig (the same count as chase_ngroups): one thread
__global__ void k_goff(int n, int b, int nb2, int *__restrict__ goff)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int nsw = n - 2;
    if (nsw <= 0) return;
    const int nsig = (nsw + nb2 - 1) / nb2;
    int tot = 0;
    for (int sg = 0; sg < nsig; ++sg) {
        goff[sg] = tot;
        tot += 1 + (n - 2 - sg * nb2) / b;
    }
    goff[nsig] = tot;
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

// Workgroups of the bulge-chase launch: enough for the sweeps that can be in
// flight at once (a sweep of n/b steps starts about every second step of its
// predecessor, so about n/(2b) are in flight) with room to spare, so that a
// sweep never waits for a free workgroup; never more than the device holds.
// The CUs left free take other streams' work meanwhile.
int chase_workgroups(int n, int b)
{
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int occ = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_bulge_chase, 256, 0);
    if (occ < 1) occ = 1;
    int G = ncu * occ;
    const int inflight = n / (2 * (b > 0 ? b : 1)) + 16;
    if (G > inflight) G = inflight;
    if (G > n - 2) G = n - 2;
    if (G < 1) G = 1;
    return G;
}

// progress: n - 2 counters and the ticket after them, all zero on entry.
hipError_t launch_chase(double *ab, int ldab, int n, int b, int nb2, double *V2, double *tau2,
                        const int *goff, unsigned *progress, unsigned *err, double *alpha, hipStream_t st)
{
    if (n >= 3) {
        int G = chase_workgroups(n, b);
        ChaseProb one{ab, V2, tau2, goff, progress, err, ldab, n, b, nb2};
        hipLaunchKernelGGL(k_bulge_chase, dim3(G), dim3(256), 0, st, one, (const ChaseProb *)nullptr,
                           (const int *)nullptr, 0, 0, progress + (n - 2));
    }
    if (n >= 2) hipLaunchKernelGGL(k_alpha, dim3(cdiv(n, 256)), dim3(256), 0, st, (const double *)ab, ldab, n, alpha);
    return hipGetLastError();
}

hipError_t launch_chase_batched(const ChaseProb *probs, const int *lanes, int M, int maxlen, int G,
                                unsigned *ticket, hipStream_t st)
{
    if (M <= 0 || maxlen <= 0) return hipSuccess;
    ChaseProb none{};
    hipLaunchKernelGGL(k_bulge_chase, dim3(G), dim3(256), 0, st, none, probs, lanes, M, maxlen, ticket);
    return hipGetLastError();
}

void launch_goff(int n, int b, int nb2, int *goff, hipStream_t st)
{
    if (n >= 3) hipLaunchKernelGGL(k_goff, dim3(1), dim3(64), 0, st, n, b, nb2, goff);
}

void launch_alpha(const double *ab, int ldab, int n, double *alpha, hipStream_t st)
{
    if (n >= 2) hipLaunchKernelGGL(k_alpha, dim3(cdiv(n, 256)), dim3(256), 0, st, ab, ldab, n, alpha);
}

int chase_max_workgroups()
{
    int dev = 0, ncu = 256, occ = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_bulge_chase, 256, 0);
    return ncu * (occ < 1 ? 1 : occ);
}

}  // namespace skew
