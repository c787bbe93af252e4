/*
 * skew_evd.h - dense real skew-symmetric eigensolver for AMD MI355X (gfx950).
 *
 * Problem (Penke, Marek, Vorwerk, Draxl, Benner, "High Performance Solution of
 * Skew-symmetric Eigenvalue Problems with Applications in Solving the
 * Bethe-Salpeter Eigenvalue Problem", Section 2.2, Algorithm 1): for a real
 * A = -A^T of order n, find real lambda_k and unitary Q with
 * Q^H A Q = diag(i lambda_k).  The eigenvalues come in pairs +-i lambda and the
 * eigenvectors of a pair are complex conjugates (Section 2.1), so only the
 * non-negative half is computed.
 *
 * Method (Sections 2.1-2.3): two-stage tridiagonalization (blocked Householder
 * full-to-band reduction with skew rank-2b updates A += V W^T - W V^T, then
 * band-to-tridiagonal bulge chasing with skew SYMV/SYR2 on the diagonal
 * blocks), the symmetric tridiagonal eigenproblem of Lemma 1, the
 * back-transformation by D = diag(i^k) and the two-stage Householder
 * back-transformation of the real and imaginary parts.
 *
 * Conventions common to every entry point:
 *  - Matrices are column-major, FP64.  A, lambda, Z_re, Z_im, alpha, band and
 *    Q arguments are DEVICE pointers (hipMalloc memory, or a PyTorch ROCm
 *    tensor's data pointer) on the current HIP device.
 *  - Only the strict lower triangle of A is read (A_ij = -A_ji); the diagonal
 *    and the upper triangle are ignored.  A is never written.
 *  - The caller owns every buffer passed in; the library never frees caller
 *    memory.  A handle owns its internal workspace (grown on demand, freed by
 *    skew_evd_destroy).
 *  - Return value: SKEW_EVD_OK (0) on success; -k when argument k (1-based,
 *    LAPACK info convention) is invalid; a positive SKEW_EVD_* code otherwise.
 *    Invalid arguments are detected before any device work is queued.
 */
#ifndef SKEW_EVD_H
#define SKEW_EVD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKEW_EVD_OK 0
#define SKEW_EVD_ERR_NONFINITE 1   /* NaN or Inf in the strict lower triangle */
#define SKEW_EVD_ERR_NOCONV 2      /* the inverse iteration of the tridiagonal solve left a vector
                                      whose residual exceeds 1e-12 ||T||, or a device-side wait
                                      did not finish */
#define SKEW_EVD_WARN_REFINE 3     /* precision form with opts.no_fp64_fallback = 1: the refinement
                                      stopped above its tolerance, or met pairs closer than its FP32
                                      start resolves; the outputs hold the last refined iterate.
                                      With the default (no_fp64_fallback = 0) such a solve is done
                                      again in the FP64 form (info->refine_sweeps = -1) instead */
#define SKEW_EVD_ERR_NOMEM 4       /* workspace allocation failed or exceeds opts.workspace_limit */
#define SKEW_EVD_ERR_HIP 5         /* HIP runtime error; text from skew_evd_status_string */
#define SKEW_EVD_ERR_NODEVICE 6    /* no usable gfx950 device */
#define SKEW_EVD_ERR_NOTDEF 7      /* skew_evd_bse: [[A, B], [conj(B), conj(A)]] is not positive
                                      definite (the Cholesky factorization of M failed) */

#define SKEW_EVD_PREC_FP64 0        /* every stage in FP64 */
#define SKEW_EVD_PREC_FP32_REFINE 1 /* band reduction and back-transformation in FP32
                                       (FP32 MFMA, FP64 norms), then FP64 refinement */
#define SKEW_EVD_PREC_BF16_REFINE 2 /* not built: refused as an argument error.  A BF16
                                       reduction starts the refinement about 0.03 from the
                                       eigenpairs at n = 16384, beyond the Newton step's reach
                                       for every pair (the FP32 start is 4.5e-7) */

typedef struct skew_evd_opts {
    int precision;          /* SKEW_EVD_PREC_*; default FP64 */
    int band;               /* semi-bandwidth b of the intermediate band matrix
                               (= panel width of the full-to-band stage); 0 = auto.
                               Supported: 8, 16, 32, 64 */
    int max_refine_sweeps;  /* precision form: refinement sweeps (default 3) */
    double refine_tol;      /* precision form: stop when the normalised
                               residual estimate is below this (default 1e-14) */
    size_t workspace_limit; /* bytes; 0 = unlimited.  Exceeding it returns NOMEM */
    int profile;            /* 1: time the main kernels with HIP events (info->kern);
                               2: time only the stage-2 application kernel */
    int autotune;           /* 1: with band = 0 and n <= SKEW_EVD_TUNE_NMAX, take the
                               band width skew_evd_autotune picks for n's size class
                               (tuned on first use, cached in the handle); 0 (default):
                               a fixed rule by n */
    int no_fp64_fallback;   /* precision form: 0 (default) = a solve whose refinement does
                               not reach refine_tol is solved again in FP64; 1 = return the
                               last iterate with SKEW_EVD_WARN_REFINE */
    int debug;              /* SKEW_EVD_DEBUG_* bits (test hooks; 0 = none) */
    int all_pairs;          /* 1: all n eigenpairs (both signs; see skew_evd_ex); 0 (default):
                               the non-negative half */
    int panel_method;       /* full-to-band panels: SKEW_EVD_PANEL_* (0 = auto: the autotuner's
                               choice with opts.autotune, else a fixed rule by n) */
    int reduction;          /* SKEW_EVD_REDUCE_TWO_STAGE (default), SKEW_EVD_REDUCE_ONE_STAGE or
                               SKEW_EVD_REDUCE_COMPLEX_HERMITIAN */
    int tridiag_method;     /* SKEW_EVD_TRIDIAG_BISECT_INVIT (0, the default and the only
                               method built); other values are argument errors */
} skew_evd_opts;

/* Symmetric tridiagonal eigensolver (Algorithm 1, step 2): multisection
 * bisection on Sturm counts and inverse iteration with Gram-Schmidt across
 * close eigenvalues (the method the paper names for its BSE runs).  The paper's
 * ELPA runs use divide and conquer, which is not built. */
#define SKEW_EVD_TRIDIAG_BISECT_INVIT 0

/* Reduction to tridiagonal form.  TWO_STAGE: full-to-band, then bulge chasing
 * (Section 2.3.2, the ELPA2 route).  ONE_STAGE (Section 2.3.1, the ELPA1 route
 * that the paper's GPU variant offloads): Householder reflectors column by
 * column, each needing a skew matrix-vector product with the whole trailing
 * matrix (streamed from HBM), the rank-2 updates of a panel of 64 columns
 * deferred to one skew rank-128 update; FP64 only, band must be 0; its
 * back-transformation is one stage of 64-reflector compact-WY blocks. */
#define SKEW_EVD_REDUCE_TWO_STAGE 0
#define SKEW_EVD_REDUCE_ONE_STAGE 1
/* COMPLEX_HERMITIAN: the comparison route of the paper's introduction and
 * Section 4.1 (Table 1): the Hermitian matrix H = iA is solved with complex
 * arithmetic as a general complex Hermitian eigensolver would, without using
 * its structure: one-stage complex Householder tridiagonalization (H held as
 * real and imaginary planes of its lower triangle; reflectors H_c = I - tau v v^H
 * with complex tau and real beta, so the tridiagonal matrix is real), the
 * eigenpairs of index floor(n/2) .. floor(n/2) + nev - 1 in ascending order of
 * that real symmetric tridiagonal matrix with its diagonal (for iA these are
 * the non-negative half, H x = lambda x), and the back-transformation by
 * complex compact-WY blocks of 64 reflectors.  The results are returned in the
 * skew solver's form: lambda and z = conj(x), A z = i lambda z.  FP64 only,
 * band must be 0.  The workspace holds both planes of H: twice the skew
 * routes' n x n. */
#define SKEW_EVD_REDUCE_COMPLEX_HERMITIAN 2

/* Panel factorization of the full-to-band stage (Section 2.3.2). */
#define SKEW_EVD_PANEL_AUTO 0
#define SKEW_EVD_PANEL_CHOLQR 1      /* Cholesky QR twice + Householder reconstruction: a few
                                        GEMM-shaped launches per panel (panels of fewer than b
                                        rows use the Householder kernel) */
#define SKEW_EVD_PANEL_HOUSEHOLDER 2 /* column-by-column Householder QR in one launch of
                                        ceil(m/128) workgroups with a grid barrier per column */

/* Debug bits of skew_evd_opts.debug (test hooks, not for production use). */
#define SKEW_EVD_DEBUG_NAN_WS 1        /* fill the handle's workspace with NaN bytes (0xFF)
                                          before the solve: results must not change */
#define SKEW_EVD_DEBUG_ZERO_WS 2       /* fill the workspace with zero bytes before the solve */
#define SKEW_EVD_DEBUG_INVIT_NOCONV 4  /* the inverse iteration's convergence test accepts no
                                          vector: the tridiagonal solve reports NOCONV */

/* Main kernels, for the per-kernel statistics of skew_evd_info. */
#define SKEW_EVD_K_PANEL 0   /* panel Householder QR (full-to-band); the whole one-stage reduction */
#define SKEW_EVD_K_SYMM 1    /* Y = A V T and W = Y - V X / 2 (full-to-band) */
#define SKEW_EVD_K_SYR2K 2   /* A += V W^T - W V^T (full-to-band) */
#define SKEW_EVD_K_CHASE 3   /* bulge chasing */
#define SKEW_EVD_K_TRIDIAG 4 /* bisection, inverse iteration, Gram-Schmidt */
#define SKEW_EVD_K_BT2 5     /* stage-2 back-transformation (the application kernel) */
#define SKEW_EVD_K_BT1 6     /* stage-1 back-transformation */
#define SKEW_EVD_K_REFINE 7  /* refinement (precision form) */
#define SKEW_EVD_NKERN 8

#define SKEW_EVD_BOUND_MFMA 0
#define SKEW_EVD_BOUND_HBM 1
#define SKEW_EVD_BOUND_ALU 2

typedef struct skew_evd_kstat {
    double ms;              /* summed device time of the kernel's launches */
    double flops;           /* algorithmic flop count of those launches */
    double bytes;           /* algorithmic HBM bytes of those launches */
    int launches;           /* number of launches timed */
    int bound;              /* SKEW_EVD_BOUND_* : the roofline that bounds it */
} skew_evd_kstat;

typedef struct skew_evd_info {
    double ms_total;        /* device time of the whole call (HIP events) */
    double ms_stage[8];     /* 0 ingest, 1 full->band, 2 bulge chase,
                               3 tridiagonal solve, 4 back-transform stage 2 (incl. D),
                               5 back-transform stage 1, 6 refinement, 7 copy-out */
    int band;               /* band width used */
    int refine_sweeps;      /* sweeps performed (precision form) */
    double refine_residual; /* last normalised residual estimate (precision form) */
    size_t workspace_bytes; /* device workspace held by the handle */
    skew_evd_kstat kern[SKEW_EVD_NKERN]; /* filled when opts.profile = 1 (only SKEW_EVD_K_BT2 with 2) */
} skew_evd_info;

typedef struct skew_evd_handle_s *skew_evd_handle;

/* Fill *opts with the defaults described above. */
void skew_evd_default_opts(skew_evd_opts *opts);

/* Create a handle bound to the current HIP device and to the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the null stream).  The handle is not
 * thread-safe; use one handle per host thread. */
int skew_evd_create(skew_evd_handle *h, void *hip_stream);
int skew_evd_destroy(skew_evd_handle h);

/* The solver (Algorithm 1; Section 2.1 for the half spectrum).
 *   n        order of A (n >= 0)
 *   A        n x n, leading dimension lda >= max(1, n); strict lower triangle read
 *   nev      number of eigenpairs, 0 <= nev <= ceil(n/2) (nev = n with all_pairs)
 *   lambda   out, nev values: the nev smallest of the ceil(n/2) values
 *            lambda >= 0 of the spectrum {+-i lambda} (plus the exact 0 of odd
 *            n, returned as lambda[0] = 0), ascending
 *   Z_re, Z_im  out, n x nev (leading dimensions ldzr, ldzi >= max(1, n)):
 *            z_k = Z_re[:,k] + i Z_im[:,k] satisfies A z_k = +i lambda_k z_k,
 *            ||z_k||_2 = 1, and the z_k are orthonormal.  conj(z_k) belongs to
 *            -i lambda_k.  The phase of each z_k is unspecified.
 *   opts     NULL = defaults
 *   info     NULL or filled after the call's device work completed
 * With opts->all_pairs = 1 (the "100 %" case of Section 4.1: every
 * eigenvector) nev must be n: lambda[0..n) receives the whole spectrum as
 * signed values mu_j ascending (A z_j = i mu_j z_j: -lambda_max .. -lambda_1,
 * then the non-negative half, the exact 0 of odd n once) and column j of
 * Z_re / Z_im the eigenvector of mu_j.  Only the non-negative half is
 * computed; the vector of -lambda_k is conj(z_k), a copy.
 * skew_evd_ex is synchronous with respect to the handle's stream: it returns
 * after the results are in Z_re/Z_im/lambda.  Argument numbers for errors:
 * -2 n, -3 A, -4 lda, -5 nev, -6 lambda, -7 Z_re, -8 ldzr, -9 Z_im, -10 ldzi,
 * -11 opts. */
int skew_evd_ex(skew_evd_handle h, int n, const double *A, int lda, int nev,
                double *lambda, double *Z_re, int ldzr, double *Z_im, int ldzi,
                const skew_evd_opts *opts, skew_evd_info *info);

/* Convenience form with ldz = n, default options, an internal handle on the
 * null stream of the current device.  Errors: -1 n, -2 A, -3 lda, -4 nev,
 * -5 lambda, -6 Z_re, -7 Z_im. */
int skew_evd(int n, const double *A, int lda, int nev,
             double *lambda, double *Z_re, double *Z_im);

/* Batched form: count independent problems (host arrays of per-problem sizes
 * and device pointers), each solved as by skew_evd_ex with ldz = n[i] (the
 * two-stage FP64 route: opts->precision and opts->reduction other than the
 * defaults return -10).
 * Problems up to n = 4096 are solved together: their stages run side by side
 * on 16 streams of the handle (HIP maps streams onto GPU_MAX_HW_QUEUES
 * hardware queues per process, 4 unless the environment sets more; 16 lets
 * them all run at once) and one bulge-chase launch serves all bands.  Their
 * launches are captured as a HIP graph on the first call of a batch
 * signature (every n, nev, band, input and output pointer and lda) and the
 * graph is replayed by later calls with the same signature, which saves the
 * host the enqueueing of each launch; the handle keeps the graph of the last
 * signature.  A replay reads the inputs present at its addresses when it
 * runs.  Larger problems, and problems whose spectrum holds a degenerate
 * cluster (flagged on the device), are solved one by one after the batch.
 * status[i] (host) receives each problem's status; the return value is the
 * first non-zero status (or a negative argument error: -2 count, -3 n,
 * -4 A, -5 lda, -6 nev, -7 lambda, -8 Z_re, -9 Z_im, -12 status).  With
 * opts->autotune, each size class is tuned on h before any problem is solved;
 * if tuning fails, no problem is solved and every status[i] holds the
 * tuner's status, which is also returned. */
int skew_evd_batched(skew_evd_handle h, int count, const int *n,
                     const double *const *A, const int *lda, const int *nev,
                     double *const *lambda, double *const *Z_re,
                     double *const *Z_im, const skew_evd_opts *opts,
                     skew_evd_info *info, int *status);

/* The Bethe-Salpeter eigenvalue problem through the skew-symmetric solver
 * (Section 3, the four steps of the BSEPACK method; Theorem 2):
 *   H_BS = [[A, B], [-conj(B), -conj(A)]],  A = A^H,  B = B^T  (m x m complex),
 * definite ([[A, B], [conj(B), conj(A)]] > 0), so its eigenvalues are real
 * pairs +-lambda.  Steps: M = [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]]
 * (Eq. SymmetricM, M = JH), Cholesky M = L L^T, eigenpairs of the skew-
 * symmetric K = L^T J L (J = [[0, I], [-I, 0]]) by skew_evd_ex, and
 * x = sqrt(lambda) Q L^{-T} z with Q = [[I, -iI], [I, iI]] / sqrt(2).
 *   m        order of A and B (m >= 0); the problem has order 2m
 *   A_re, A_im   real and imaginary planes of A (m x m, column-major, lda >= m);
 *            the real plane is read in its lower triangle (diagonal included),
 *            the imaginary plane entirely
 *   B_re, B_im   the same for B (ldb >= m)
 *   nev      0 <= nev <= m: the nev smallest positive eigenvalues
 *   lambda   out, nev values, ascending
 *   X_re, X_im   out, 2m x nev (ldx >= 2m): H_BS x_k = lambda_k x_k with the
 *            BSE normalization x_k^H S x_k = 1, S = diag(I_m, -I_m); the
 *            vector of -lambda_k is [conj(v); conj(u)] for x_k = [u; v]
 *   opts     as for skew_evd_ex (precision, band, panel method, ...) for the
 *            skew-symmetric eigenproblem; all_pairs must be 0
 * Device pointers; synchronous with respect to h's stream; the handle holds a
 * second workspace for M (then L), K and the back-transformation, about
 * 8 (8 m^2 + 4 m nev + 4096 nev) bytes, grown on demand.
 * Errors: -1 h, -2 m, -3 A_re, -4 A_im, -5 lda, -6 B_re, -7 B_im, -8 ldb,
 * -9 nev, -10 lambda, -11 X_re, -12 X_im, -13 ldx, -14 opts;
 * SKEW_EVD_ERR_NONFINITE (a NaN or Inf among the entries of M),
 * SKEW_EVD_ERR_NOTDEF, or a status of skew_evd_ex. */
int skew_evd_bse(skew_evd_handle h, int m, const double *A_re, const double *A_im, int lda,
                 const double *B_re, const double *B_im, int ldb, int nev, double *lambda,
                 double *X_re, double *X_im, int ldx, const skew_evd_opts *opts,
                 skew_evd_info *info);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The FP64 solver of skew_evd_ex with default options for orders
 * n <= SKEW_EVD_NOALLOC_NMAX, on the HIP stream `hip_stream` (a hipStream_t,
 * NULL = the null stream) of the current device; arguments as for skew_evd_ex
 * (device pointers; only the strict lower triangle of A is read).  It calls no
 * hipMalloc, hipFree, hipHostMalloc or event/stream creation: its workspace is
 * a fixed device array of SKEW_EVD_NOALLOC_BYTES bytes that the library holds
 * on every device it runs on until the process ends, and its host-side state
 * is fixed storage, one slot per device.  Every call on a device shares that
 * device's array, which keeps the last call's contents (every call clears what
 * it needs cleared), so calls that overlap on one device -- from several host
 * threads or streams -- race and must be serialized by the caller.
 * Synchronous with respect to hip_stream: it returns after the results are in
 * lambda / Z_re / Z_im (it reads status words back, so it cannot itself be
 * captured in a graph).
 * Errors: -1 n, -2 A, -3 lda, -4 nev, -5 lambda, -6 Z_re, -7 ldzr, -8 Z_im,
 * -9 ldzi; SKEW_EVD_ERR_NOMEM (before any device work) when
 * n > SKEW_EVD_NOALLOC_NMAX; otherwise the statuses of skew_evd_ex. */
#define SKEW_EVD_NOALLOC_NMAX 512
#define SKEW_EVD_NOALLOC_BYTES (48u << 20)
int skew_evd_noalloc(int n, const double *A, int lda, int nev, double *lambda,
                     double *Z_re, int ldzr, double *Z_im, int ldzi, void *hip_stream);

/* Stage entry points (building blocks, also used by the stage-level tests). */

/* Full-to-band reduction (Section 2.3.2): B = Q_band^T A Q_band with semi-
 * bandwidth b.  band: (b+1) x n column-major, ldband >= b+1, LAPACK lower band
 * storage: band[d + j*ldband] = B[j+d, j], d = 0..b (the diagonal row d = 0 is
 * written as 0).  Errors: -2 n, -3 A, -4 lda, -5 b, -6 band, -7 ldband. */
int skew_evd_band_reduce(skew_evd_handle h, int n, const double *A, int lda,
                         int b, double *band, int ldband);

/* Two-stage tridiagonalization (Algorithm 1, step 1): alpha[j] = A_trd[j, j+1],
 * j = 0..n-2 (the super-diagonal; the sub-diagonal is -alpha).
 * Errors: -2 n, -3 A, -4 lda, -5 b, -6 alpha. */
int skew_evd_tridiagonalize(skew_evd_handle h, int n, const double *A, int lda,
                            int b, double *alpha);

/* Symmetric tridiagonal eigensolve (Algorithm 1, step 2, Lemma 1):
 * T = tridiag(alpha, 0, alpha) of order n; lambda[0..nev) = its eigenvalues
 * with ascending indices floor(n/2)..floor(n/2)+nev-1 (the non-negative half),
 * Q (n x nev, ldq >= n) the orthonormal eigenvectors.
 * Errors: -2 n, -3 alpha, -4 nev, -5 lambda, -6 Q, -7 ldq. */
int skew_evd_tridiag_eig(skew_evd_handle h, int n, const double *alpha, int nev,
                         double *lambda, double *Q, int ldq);

/* Band-width and panel-method autotuner (not in the paper; Section 4.1 notes
 * how strongly the speed of a reduction can depend on its block size).  Orders
 * are grouped in size classes of 128 (n in (128(c-1), 128c]).  On the first
 * call for a class and precision, a seeded synthetic skew matrix of order 128c
 * (entries (u - u')/2 with u, u' independent and uniform in [-1, 1)) is solved
 * on h's stream once per candidate: band width {16, 32, 64} times panel method
 * {SKEW_EVD_PANEL_CHOLQR, SKEW_EVD_PANEL_HOUSEHOLDER}, one warm-up and three
 * timed calls each, host wall clock.  The fastest pair is cached in h (solves
 * with opts.autotune use both); its band is returned in *band and *ms (may be
 * NULL) receives its best time per solve in milliseconds.  Later calls for the class return the cached values without
 * solving.  Tuning allocates and frees its own device buffers (an input and
 * outputs of order 128c) and grows h's workspace.
 *   n          1 <= n <= SKEW_EVD_TUNE_NMAX
 *   precision  SKEW_EVD_PREC_FP64 or SKEW_EVD_PREC_FP32_REFINE
 * Errors: -1 h, -2 n, -3 precision, -4 band; SKEW_EVD_ERR_NOMEM if the tuning
 * buffers cannot be allocated; a solver status if every candidate failed. */
#define SKEW_EVD_TUNE_NMAX 8192
int skew_evd_autotune(skew_evd_handle h, int n, int precision, int *band,
                      double *ms);

/* Text for a status code (static storage; for SKEW_EVD_ERR_HIP the text of the
 * most recent HIP error seen by this thread). */
const char *skew_evd_status_string(int status);

/* Library version, major*10000 + minor*100 + patch. */
int skew_evd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SKEW_EVD_H */
