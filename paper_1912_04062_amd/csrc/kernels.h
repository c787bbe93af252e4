// Host-side launchers of the device kernels (internal interface between the
// stage drivers in api.cpp and the kernel files).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace skew {

// band.hip
void launch_fill32(void *p, unsigned v, size_t nwords, hipStream_t st);
template <typename T>
void launch_ingest(const double *A, int lda, int n, T *W, int ldw, unsigned *flags, hipStream_t st);
int panel_qr_groups(int m);
size_t panel_qr_part_doubles(int m, int B);
template <typename T>
hipError_t launch_panel_qr(T *W, int ldw, int c0, int r0, int m, int B, T *Vd, double *tau, double *Tf,
                           double *part, unsigned *bar, unsigned bar_base, unsigned *err, const unsigned *skip,
                           hipStream_t st);
// Cholesky-QR panel path (FP64): Gram partial reduction, Cholesky step
// (pass 1 or 2, sets *flag when the panel needs the Householder kernel),
// Householder reconstruction; scratch cq of cholqr_scratch_doubles().
constexpr int CQ_G = 0, CQ_R1 = 1, CQ_R1INV = 2, CQ_R2INV = 3, CQ_R = 4, CQ_UINV = 5;
size_t cholqr_scratch_doubles();
void launch_gram_reduce(const double *Gp, int np, int BB, double *G, hipStream_t st);
// Gp non-null: the Gram matrix is the sum of its np partials (summed here)
void launch_chol_qr(int B, int pass, double *cq, unsigned *flag, hipStream_t st, const double *Gp = nullptr,
                    int np = 0);
template <typename T>
void launch_hh_rebuild(T *Vd, int m, int B, T *Wp, int ldw, double *cq, double *Tf, double *tau,
                       const unsigned *flag, hipStream_t st);
int symm_splits(int m);
int symm_kchunk(int m, int S);
int gram_chunk_rows();
template <typename T>
void launch_stage1_w(T *W, int ldw, int r0, int m, int B, const T *Vd, const double *Tf, T *Ypart,
                     T *Y0, T *Wd, double *Gp, T *Tx, hipStream_t st);
template <typename T>
void launch_stage1_syr2k(T *W, int ldw, int r0, int m, int B, const T *Vd, const T *Wd, hipStream_t st);
// the same with V and W of leading dimension ldv (>= m)
template <typename T>
void launch_syr2k_ld(T *W, int ldw, int r0, int m, int B, const T *Vd, const T *Wd, int ldv, hipStream_t st);
template <typename T>
void launch_band_extract(const T *W, int ldw, int n, int b, double *ab, int ldab, hipStream_t st);

// chase.hip
int chase_ngroups(int n, int b, int nb2, int *goff_host);
hipError_t launch_chase(double *ab, int ldab, int n, int b, int nb2, double *V2, double *tau2,
                        const int *goff, unsigned *progress, unsigned *err, double *alpha, hipStream_t st);
// one band of a batched chase (device array of these); progress: n - 2 zeroed counters
struct ChaseProb {
    double *ab, *V2, *tau2;
    const int *goff;
    unsigned *progress, *err;
    int ldab, n, b, nb2;
};
// lanes: [M + 1] item ranges per lane, then per item (problem, first position
// in its lane); maxlen = longest lane in sweeps; G workgroups; *ticket zeroed
hipError_t launch_chase_batched(const ChaseProb *probs, const int *lanes, int M, int maxlen, int G,
                                unsigned *ticket, hipStream_t st);
void launch_alpha(const double *ab, int ldab, int n, double *alpha, hipStream_t st);
int chase_max_workgroups();
// group offsets of the stage-2 reflectors, computed on the device (nsig + 1 entries)
void launch_goff(int n, int b, int nb2, int *goff, hipStream_t st);

// tridiag.hip
// diag: the diagonal of a general symmetric tridiagonal matrix (n entries),
// or null for the zero diagonal of Lemma 1
// gcnt: tri_grid_points(count) ints for the grid pre-pass (null: none)
void launch_tridiag_eigvals(const double *alpha, int n, int first, int count, double *a2, double *stats,
                            double *w, hipStream_t st, const double *diag = nullptr, int *gcnt = nullptr);
int tri_grid_points(int nev);
void launch_tridiag_eigvecs(const double *alpha, int n, int nev, const double *w, const double *stats,
                            double *U0, double *U1, double *U2, double *Lm, unsigned char *Sw, double *Y,
                            double *fac, double *Q, int ldq, double ctol, unsigned *err, hipStream_t st,
                            const double *diag = nullptr);
void launch_tridiag_polish(const double *alpha, int n, int m, const double *w, const double *shifts,
                           const double *stats, double *U0, double *U1, double *U2, double *Lm, unsigned char *Sw,
                           double *Y, double *fac, double *Q, int ldq, hipStream_t st, const double *diag = nullptr);
// One tridiagonal problem of the batched eigenvalue and eigenvector launches
// (device pointers into the problem's workspace; ab: its band, from which
// alpha is extracted first).  first: index of the first eigenvalue (n / 2),
// nev: eigenpairs, iters: inverse-iteration steps, ctol: its residual test.
struct TriProb {
    const double *ab;
    double *alpha, *a2, *stats, *w;
    double *U0, *U1, *U2, *Lm, *Y, *fac, *Q;
    unsigned char *Sw;
    unsigned *err;
    int *gcnt;                  // counts of the bisection's grid pre-pass (null: none)
    const double *diag, *shifts;
    double ctol;
    int ldab, n, first, nev, ldq, iters;
};
// Workgroups per problem of the batched launches (prefix tables over the
// problems, cnt + 1 entries each, in this order in `pre`).
int tri_bisect_groups(int nev);
int tri_invit_groups(int nev);
int tri_transpose_groups(int n, int nev);
// alpha from the band, alpha^2 and the norms, eigenvalues, eigenvectors (with
// the odd-order null vector) into each problem's Q: one launch per kernel for
// all cnt problems; tot[t] = pre table t's last entry
void launch_tridiag_batched(const TriProb *probs, const int *pre, int cnt, const int tot[3], hipStream_t st);
// sets *flag when two consecutive values of w[0..m) are closer than tol * stats[0]
void launch_degenerate_check(const double *w, int m, const double *stats, double tol, unsigned *flag,
                             hipStream_t st);
void launch_chol_inv(const double *Gp, int nparts, int NB, double *Rinv, hipStream_t st);

// backtransform.hip
// launch_bt2 phases: bit 0 = T factors of the reflector groups, bit 1 = application.
template <typename T>
void launch_dscale(const double *Q, int ldq, int n, int nev, T *Z, int ldz, hipStream_t st);
template <typename T>
void launch_bt2(T *Z, int ldz, int n, int ncols, int b, int nb2, const double *V2, const double *tau2, T *T2,
                T *V2t, const int *goff_dev, int nsig, int ngroups, int phases,
                hipStream_t st);
int tn_splits(int K, int tiles);
template <typename T>
int launch_gemm_tn_part(const T *A, int lda, const T *B, int ldb, int M, int N, int K, double *Cpart,
                        hipStream_t st, int S_req = 0);
// the same for FP32 operands with FP64 products and sums
int launch_gemm_tn_part_f64(const float *A, int lda, const float *B, int ldb, int M, int N, int K, double *Cpart,
                            hipStream_t st, int S_req = 0);
template <typename T>
void launch_gemm_nn(const T *A, int lda, const double *Bpart, int S, int M, int N, int K, T *C, int ldc,
                    double alpha, int beta, hipStream_t st);
void launch_reduce_left(const double *S0, const double *Cpart, int S, int M, int N, double *out,
                        hipStream_t st);
template <typename T>
void launch_copy_cols(const T *src, int lds, T *dst, int ldd, int m, int ncol, hipStream_t st);
void launch_to_float(const double *src, int lds, float *dst, int ldd, int m, int ncol, hipStream_t st);
// columns c < off <- conj(column n-1-c), lam[c] = -lam[n-1-c] (whole-spectrum output)
void launch_mirror(double *Zr, int ldr, double *Zi, int ldi, double *lam, int n, int off, hipStream_t st);
template <typename T>
void launch_to_double(const T *src, int lds, double *dst, int ldd, int m, int ncol, hipStream_t st);

// Stage-1 block Z[r0:r0+m, 0:ncols] -= V T V^T Z[r0:r0+m, :] for KK in {32, 64, 128}
// reflectors (V = [V1, V2 shifted by b1 rows] when V2 is given).  Wp holds
// bt1_max_splits() * KK * ncols doubles, W2 KK * ncols elements.
constexpr int bt1_max_splits() { return 16; }
int bt1_splits(int m, int ncols);
template <typename T>
void launch_bt1_block(T *Z, int ldz, int r0, int m, int ncols, const T *V1, int b1, const T *V2, int m2,
                      const double *Tm, int KK, double *Wp, T *W2, hipStream_t st);
void launch_merge_t(const double *T1, const double *T2, const double *Gp, int S, int b, double *Tm, hipStream_t st);

// onestage.hip (one-stage tridiagonalization)
size_t onestage_scratch_doubles(int n);
void launch_onestage_panel(double *A, int lda, int n, int c0, int nb, double *V, double *W, int ldv, double *tau,
                           double *T, double *alpha, double *scratch, hipStream_t st);

// hermitian.hip (the complex Hermitian route on iA)
size_t herm_scratch_doubles(int n);
void launch_herm_panel(double *Hr, double *Hi, int lda, int n, int c0, int nb, double *Vr, double *Vi, double *Wr,
                       double *Wi, int ldv, double *tau, double *Tr, double *Ti, double *d, double *e,
                       double *scratch, hipStream_t st);
void launch_herm_bt(double *Z, int ldz, int r0, int m, int nev, const double *Vr, const double *Vi, const double *Tr,
                    const double *Ti, double *P1, double *P2, double *B, hipStream_t st);
void launch_negate(double *X, size_t count, hipStream_t st);

// bse.hip (the Bethe-Salpeter route)
void launch_bse_build_m(const double *Ar, const double *Ai, int lda, const double *Br, const double *Bi, int ldb,
                        int m, double *M, int ldm, unsigned *flags, hipStream_t st);
// blocked Cholesky of the lower triangle of M (n x n) in place; R^{-1} of each
// diagonal block (64 x 64) into Rinv_all; bit 4 of *flags when M is not
// positive definite
void launch_cholesky(double *M, int ldm, int n, double *Rinv_all, unsigned *flags, hipStream_t st);
void launch_ltjl(const double *L, int ldl, int m, double *K, int ldk, hipStream_t st);
// Z <- L^{-T} Z (n x ncols), Wp: tn_parts_max x 64 x ncols doubles
void launch_trsm_lt(const double *L, int ldl, int n, const double *Rinv_all, double *Z, int ldz, int ncols,
                    double *Wp, hipStream_t st);
void launch_bse_x(const double *Z, int ldz, int m, int nev, const double *lam, double *Xr, double *Xi, int ldx,
                  hipStream_t st);

// refine.hip
template <typename T>
void launch_build_x(const T *Z, int ldz, int n, int nev, int odd, double *X, hipStream_t st);
void launch_split_x(const double *X, int n, int nev, int odd, double *Zr, int ldr, double *Zi, int ldi,
                    hipStream_t st);
void launch_refine_products(const double *A, int lda, int n, const double *X, int ncx, double *P, double *S,
                            double *G, hipStream_t st);
void launch_refine_eigs(const double *S, const double *G, int ncx, int nblk, int odd, double *lam, double *stat,
                        hipStream_t st);
void launch_refine_update(const double *S, const double *G, int n, int ncx, int nblk, int odd, const double *lam,
                          double omega, float *E, const double *X, double *Xn, unsigned *nclust, double *emax,
                          hipStream_t st);

}  // namespace skew
