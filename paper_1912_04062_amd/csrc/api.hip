// C-ABI of the skew-symmetric eigensolver and the host-side stage drivers.
// The host only validates arguments, plans the workspace and enqueues kernels
// on the handle's stream; every arithmetic step runs in the device kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <vector>

#include "../../include/skew_evd.h"
#include "kernels.h"

namespace {

thread_local char g_errtext[512] = "";

void set_hip_error(hipError_t e, const char *what)
{
    snprintf(g_errtext, sizeof(g_errtext), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
}

#define HCHK(expr)                                       \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            set_hip_error(e_, #expr);                    \
            return SKEW_EVD_ERR_HIP;                     \
        }                                                \
    } while (0)

constexpr int NSTAGE_EV = 9;
constexpr int ORTH_NB = 64;

struct Plan {
    int n = 0, nev = 0, b = 0, nb2 = 0, prec = 0;
    int npanels = 0, ngroups = 0, nsig = 0;
    int orth_window = 0;
};

}  // namespace

struct skew_evd_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ev[NSTAGE_EV] = {};
    unsigned *ctl_host = nullptr;   // pinned copy of the control words
};

namespace {

// ---------------------------------------------------------------------------
// Workspace layout.  Offsets are 256-byte aligned.
struct Layout {
    size_t W, Vall, Tall, tauall, Ypart, Y0, Wd, Gp, Tx, part, ab, goff, V2, tau2, T2, V2t, alpha, a2, stats,
        lam, U0, U1, U2, Lm, Sw, Yiv, Qd, Z, Wp, Wt2, Pp, P, Gp2, Rinv, Tmp, ctl, total;
    std::vector<size_t> Voff;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int tn_parts_max() { return 32; }

Layout plan_layout(const Plan &p)
{
    Layout L;
    const size_t n = p.n, nev = p.nev, b = p.b, nb2 = p.nb2;
    const size_t es = p.prec ? sizeof(float) : sizeof(double);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al(bytes ? bytes : 1);
        return o;
    };
    L.W = take(es * n * n);
    L.Voff.clear();
    size_t vtot = 0;
    for (int j = 0; j < p.npanels; ++j) {
        L.Voff.push_back(vtot);
        size_t m = n - (size_t)(j + 1) * b;
        vtot += m * b;
    }
    L.Vall = take(es * vtot);
    L.Tall = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * b * b);
    L.tauall = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * b);
    const size_t m0 = n > b ? n - b : 1;
    L.Ypart = take(es * 16 * m0 * b);
    L.Y0 = take(es * m0 * b);
    L.Wd = take(es * m0 * b);
    L.Gp = take(sizeof(double) * (m0 / 512 + 2) * b * b);
    L.Tx = take(es * 2 * b * b);
    L.part = take(sizeof(double) * skew::panel_qr_part_doubles((int)m0, (int)b));
    L.ab = take(sizeof(double) * (2 * b + 1) * n);
    L.goff = take(sizeof(int) * (p.nsig + 2));
    L.V2 = take(sizeof(double) * (size_t)p.ngroups * b * nb2);
    L.tau2 = take(sizeof(double) * (size_t)p.ngroups * nb2);
    L.T2 = take(es * (size_t)p.ngroups * nb2 * nb2);
    L.V2t = p.prec ? take(es * (size_t)p.ngroups * b * nb2) : 0;
    L.alpha = take(sizeof(double) * n);
    L.a2 = take(sizeof(double) * n);
    L.stats = take(sizeof(double) * 4);
    L.lam = take(sizeof(double) * nev);
    L.U0 = take(sizeof(double) * n * nev);
    L.U1 = take(sizeof(double) * n * nev);
    L.U2 = take(sizeof(double) * n * nev);
    L.Lm = take(sizeof(double) * n * nev);
    L.Sw = take(n * nev);
    L.Yiv = take(sizeof(double) * n * nev);
    L.Qd = take(sizeof(double) * n * nev);
    L.Z = take(es * n * 2 * nev);
    L.Wp = take(sizeof(double) * tn_parts_max() * b * 2 * nev);
    L.Wt2 = take(sizeof(double) * b * 2 * nev);
    const size_t wmax = std::max((size_t)p.orth_window, (size_t)ORTH_NB);
    L.Pp = take(sizeof(double) * tn_parts_max() * wmax * ORTH_NB);
    L.P = take(sizeof(double) * wmax * ORTH_NB);
    L.Gp2 = take(sizeof(double) * tn_parts_max() * ORTH_NB * ORTH_NB);
    L.Rinv = take(sizeof(double) * ORTH_NB * ORTH_NB);
    L.Tmp = take(sizeof(double) * n * ORTH_NB);
    L.ctl = take(sizeof(unsigned) * (64 + n));
    L.total = off;
    return L;
}

// control words
enum { CTL_FLAGS = 0, CTL_ERR = 1, CTL_BAR = 2, CTL_PROGRESS = 64 };

int auto_band(int n)
{
    if (n >= 2048) return 64;
    if (n >= 128) return 32;
    return 16;
}

Plan make_plan(int n, int nev, int b, int prec)
{
    Plan p;
    p.n = n;
    p.nev = nev;
    p.prec = prec;
    p.b = b > 0 ? b : auto_band(n);
    p.nb2 = p.b;
    p.npanels = 0;
    for (int c0 = 0; c0 + p.b < n - 1; c0 += p.b) ++p.npanels;
    p.nsig = n > 2 ? (n - 2 + p.nb2 - 1) / p.nb2 : 0;
    p.ngroups = skew::chase_ngroups(n, p.b, p.nb2, nullptr);
    p.orth_window = nev <= 2048 ? nev : 1024;
    return p;
}

int ensure_ws(skew_evd_handle h, size_t bytes, size_t limit)
{
    if (limit && bytes > limit) {
        snprintf(g_errtext, sizeof(g_errtext), "workspace of %zu bytes exceeds the limit of %zu", bytes, limit);
        return SKEW_EVD_ERR_NOMEM;
    }
    if (bytes <= h->ws_bytes) return SKEW_EVD_OK;
    if (h->ws) {
        HCHK(hipStreamSynchronize(h->stream));
        HCHK(hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    hipError_t e = hipMalloc((void **)&h->ws, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        snprintf(g_errtext, sizeof(g_errtext), "hipMalloc of %zu bytes failed", bytes);
        return SKEW_EVD_ERR_NOMEM;
    }
    h->ws_bytes = bytes;
    return SKEW_EVD_OK;
}

template <typename T> T *ptr(skew_evd_handle h, size_t off) { return (T *)(h->ws + off); }

// ---------------------------------------------------------------------------
// Stage drivers.  All enqueue on h->stream.

template <typename T>
int stage_band(skew_evd_handle h, const Plan &p, const Layout &L, const double *A, int lda, int check_finite)
{
    hipStream_t st = h->stream;
    const int n = p.n, b = p.b;
    T *W = ptr<T>(h, L.W);
    unsigned *ctl = ptr<unsigned>(h, L.ctl);
    skew::launch_ingest<T>(A, lda, n, W, n, ctl + CTL_FLAGS, st);
    HCHK(hipGetLastError());
    if (check_finite) {
        HCHK(hipMemcpyAsync(h->ctl_host, ctl, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        if (h->ctl_host[CTL_FLAGS] & 1u) return SKEW_EVD_ERR_NONFINITE;
    }
    HCHK(hipEventRecord(h->ev[1], st));
    unsigned bar_base = 0;
    for (int j = 0; j < p.npanels; ++j) {
        const int c0 = j * b, r0 = c0 + b, m = n - r0;
        T *Vd = ptr<T>(h, L.Vall) + L.Voff[j];
        double *Tf = ptr<double>(h, L.Tall) + (size_t)j * b * b;
        HCHK(skew::launch_panel_qr<T>(W, n, c0, r0, m, b, Vd, ptr<double>(h, L.tauall) + (size_t)j * b, Tf,
                                      ptr<double>(h, L.part), ctl + CTL_BAR, bar_base, ctl + CTL_ERR, st));
        bar_base += (unsigned)((std::min(m, b) + 1) * skew::panel_qr_groups(m));
        if (m > 1)
            skew::launch_stage1_update<T>(W, n, r0, m, b, Vd, Tf, ptr<T>(h, L.Ypart), ptr<T>(h, L.Y0),
                                          ptr<T>(h, L.Wd), ptr<double>(h, L.Gp), ptr<T>(h, L.Tx), st);
        HCHK(hipGetLastError());
    }
    skew::launch_band_extract<T>(W, n, n, b, ptr<double>(h, L.ab), 2 * b + 1, st);
    HCHK(hipGetLastError());
    HCHK(hipEventRecord(h->ev[2], st));
    return SKEW_EVD_OK;
}

int stage_chase(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, b = p.b;
    std::vector<int> goff(p.nsig + 2, 0);
    skew::chase_ngroups(n, b, p.nb2, goff.data());
    HCHK(hipMemcpyAsync(ptr<int>(h, L.goff), goff.data(), sizeof(int) * (p.nsig + 1), hipMemcpyHostToDevice, st));
    if (p.ngroups > 0) {
        HCHK(hipMemsetAsync(ptr<double>(h, L.V2), 0, sizeof(double) * (size_t)p.ngroups * b * p.nb2, st));
        HCHK(hipMemsetAsync(ptr<double>(h, L.tau2), 0, sizeof(double) * (size_t)p.ngroups * p.nb2, st));
    }
    unsigned *ctl = ptr<unsigned>(h, L.ctl);
    HCHK(hipMemsetAsync(ctl + CTL_PROGRESS, 0, sizeof(unsigned) * n, st));
    HCHK(skew::launch_chase(ptr<double>(h, L.ab), 2 * b + 1, n, b, p.nb2, ptr<double>(h, L.V2),
                            ptr<double>(h, L.tau2), ptr<int>(h, L.goff), ctl + CTL_PROGRESS, ctl + CTL_ERR,
                            ptr<double>(h, L.alpha), st));
    // the goff host vector must outlive the async copy
    HCHK(hipStreamSynchronize(st));
    HCHK(hipEventRecord(h->ev[3], st));
    return SKEW_EVD_OK;
}

// Block Gram-Schmidt in eigenvalue order (window of earlier vectors, then a
// Cholesky-QR of the block).
int orthogonalize(skew_evd_handle h, const Plan &p, const Layout &L, double *Q, int ldq, int n, int nev)
{
    hipStream_t st = h->stream;
    for (int b0 = 0; b0 < nev; b0 += ORTH_NB) {
        const int nb = std::min(ORTH_NB, nev - b0);
        const int w0 = std::max(0, b0 - p.orth_window);
        const int wl = b0 - w0;
        double *Qb = Q + (size_t)b0 * ldq;
        if (wl > 0) {
            const double *Qw = Q + (size_t)w0 * ldq;
            int S = skew::launch_gemm_tn_part<double>(Qw, ldq, Qb, ldq, wl, nb, n, ptr<double>(h, L.Pp), st);
            skew::launch_reduce_left(nullptr, ptr<double>(h, L.Pp), S, wl, nb, ptr<double>(h, L.P), st);
            skew::launch_gemm_nn<double>(Qw, ldq, ptr<double>(h, L.P), 1, n, nb, wl, Qb, ldq, -1.0, 1, st);
        }
        int S = skew::launch_gemm_tn_part<double>(Qb, ldq, Qb, ldq, nb, nb, n, ptr<double>(h, L.Gp2), st);
        skew::launch_chol_inv(ptr<double>(h, L.Gp2), S, nb, ptr<double>(h, L.Rinv), st);
        skew::launch_gemm_nn<double>(Qb, ldq, ptr<double>(h, L.Rinv), 1, n, nb, nb, ptr<double>(h, L.Tmp), n, 1.0, 0,
                                     st);
        skew::launch_copy_cols<double>(ptr<double>(h, L.Tmp), n, Qb, ldq, n, nb, st);
        HCHK(hipGetLastError());
    }
    return SKEW_EVD_OK;
}

int stage_tridiag(skew_evd_handle h, const Plan &p, const Layout &L, const double *alpha, int nev, double *lam,
                  double *Q, int ldq)
{
    hipStream_t st = h->stream;
    const int n = p.n;
    skew::launch_tridiag_eigvals(alpha, n, n / 2, nev, ptr<double>(h, L.a2), ptr<double>(h, L.stats), lam, st);
    skew::launch_tridiag_eigvecs(alpha, n, nev, lam, ptr<double>(h, L.stats), ptr<double>(h, L.U0),
                                 ptr<double>(h, L.U1), ptr<double>(h, L.U2), ptr<double>(h, L.Lm),
                                 ptr<unsigned char>(h, L.Sw), ptr<double>(h, L.Yiv), Q, ldq, st);
    HCHK(hipGetLastError());
    int rc = orthogonalize(h, p, L, Q, ldq, n, nev);
    if (rc) return rc;
    HCHK(hipEventRecord(h->ev[4], st));
    return SKEW_EVD_OK;
}

template <typename T>
int stage_backtransform(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, nev = p.nev, b = p.b;
    T *Z = ptr<T>(h, L.Z);
    skew::launch_dscale<T>(ptr<double>(h, L.Qd), n, n, nev, Z, n, st);
    skew::launch_bt2<T>(Z, n, n, 2 * nev, b, p.nb2, ptr<double>(h, L.V2), ptr<double>(h, L.tau2), ptr<T>(h, L.T2),
                        p.prec ? ptr<T>(h, L.V2t) : nullptr, ptr<int>(h, L.goff), p.nsig, p.ngroups, st);
    HCHK(hipGetLastError());
    HCHK(hipEventRecord(h->ev[5], st));
    for (int j = p.npanels - 1; j >= 0; --j) {
        const int r0 = (j + 1) * b, m = n - r0;
        const T *Vd = ptr<T>(h, L.Vall) + L.Voff[j];
        const double *Tf = ptr<double>(h, L.Tall) + (size_t)j * b * b;
        int S = skew::launch_gemm_tn_part<T>(Vd, m, Z + r0, n, b, 2 * nev, m, ptr<double>(h, L.Wp), st);
        skew::launch_reduce_left(Tf, ptr<double>(h, L.Wp), S, b, 2 * nev, ptr<double>(h, L.Wt2), st);
        skew::launch_gemm_nn<T>(Vd, m, ptr<double>(h, L.Wt2), 1, m, 2 * nev, b, Z + r0, n, -1.0, 1, st);
        HCHK(hipGetLastError());
    }
    HCHK(hipEventRecord(h->ev[6], st));
    return SKEW_EVD_OK;
}

int finish_status(skew_evd_handle h, const Layout &L)
{
    unsigned *ctl = ptr<unsigned>(h, L.ctl);
    HCHK(hipMemcpyAsync(h->ctl_host, ctl, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    if (h->ctl_host[CTL_ERR]) {
        snprintf(g_errtext, sizeof(g_errtext), "a device-side wait gave up (code %u)", h->ctl_host[CTL_ERR]);
        return SKEW_EVD_ERR_NOCONV;
    }
    return SKEW_EVD_OK;
}

int check_device()
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        snprintf(g_errtext, sizeof(g_errtext), "no HIP device");
        return SKEW_EVD_ERR_NODEVICE;
    }
    return SKEW_EVD_OK;
}

int validate_opts(const skew_evd_opts *o)
{
    if (!o) return 0;
    if (o->precision != SKEW_EVD_PREC_FP64 && o->precision != SKEW_EVD_PREC_FP32_REFINE) return 1;
    if (o->band != 0 && (o->band < 8 || o->band > 64 || (o->band % 8) != 0)) return 1;
    if (o->max_refine_sweeps < 0) return 1;
    return 0;
}

int solve(skew_evd_handle h, int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr,
          double *Z_im, int ldzi, const skew_evd_opts *opts, skew_evd_info *info)
{
    skew_evd_opts o;
    skew_evd_default_opts(&o);
    if (opts) o = *opts;
    const int prec = o.precision;
    if (prec != SKEW_EVD_PREC_FP64) {
        snprintf(g_errtext, sizeof(g_errtext), "precision form not available in this build");
        return -11;
    }
    Plan p = make_plan(n, nev, o.band, prec);
    Layout L = plan_layout(p);
    int rc = ensure_ws(h, L.total, o.workspace_limit);
    if (rc) return rc;
    hipStream_t st = h->stream;
    bool rec[NSTAGE_EV] = {};
    HCHK(hipMemsetAsync(ptr<unsigned>(h, L.ctl), 0, sizeof(unsigned) * 64, st));
    HCHK(hipEventRecord(h->ev[0], st));
    rec[0] = true;
    rc = stage_band<double>(h, p, L, A, lda, 1);
    if (rc) return rc;
    rec[1] = rec[2] = true;
    rc = stage_chase(h, p, L);
    if (rc) return rc;
    rec[3] = true;
    rc = stage_tridiag(h, p, L, ptr<double>(h, L.alpha), nev, ptr<double>(h, L.lam), ptr<double>(h, L.Qd), n);
    if (rc) return rc;
    rec[4] = true;
    rc = stage_backtransform<double>(h, p, L);
    if (rc) return rc;
    rec[5] = rec[6] = true;
    HCHK(hipEventRecord(h->ev[7], st));
    rec[7] = true;
    HCHK(hipMemcpyAsync(lambda, ptr<double>(h, L.lam), sizeof(double) * nev, hipMemcpyDeviceToDevice, st));
    const double *Z = ptr<double>(h, L.Z);
    HCHK(hipMemcpy2DAsync(Z_re, sizeof(double) * ldzr, Z, sizeof(double) * n, sizeof(double) * n, nev,
                          hipMemcpyDeviceToDevice, st));
    HCHK(hipMemcpy2DAsync(Z_im, sizeof(double) * ldzi, Z + (size_t)nev * n, sizeof(double) * n,
                          sizeof(double) * n, nev, hipMemcpyDeviceToDevice, st));
    HCHK(hipEventRecord(h->ev[8], st));
    rec[8] = true;
    rc = finish_status(h, L);
    // stage slots: 0 ingest, 1 band, 2 chase, 3 tridiag, 4 BT2(+D), 5 BT1, 6 refine (none), 7 copy-out
    if (info) {
        memset(info, 0, sizeof(*info));
        info->band = p.b;
        info->workspace_bytes = h->ws_bytes;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[0], h->ev[8]) == hipSuccess) info->ms_total = ms;
        const int a[8] = {0, 1, 2, 3, 4, 5, 6, 7}, bnd[8] = {1, 2, 3, 4, 5, 6, 6, 8};
        for (int s = 0; s < 8; ++s) {
            if (s == 6) continue;
            if (hipEventElapsedTime(&ms, h->ev[a[s] == 7 ? 7 : a[s]], h->ev[bnd[s]]) == hipSuccess)
                info->ms_stage[s] = ms;
        }
    }
    return rc;
}

}  // namespace

// ===========================================================================
extern "C" {

void skew_evd_default_opts(skew_evd_opts *opts)
{
    if (!opts) return;
    memset(opts, 0, sizeof(*opts));
    opts->precision = SKEW_EVD_PREC_FP64;
    opts->band = 0;
    opts->max_refine_sweeps = 2;
    opts->refine_tol = 1e-14;
    opts->workspace_limit = 0;
}

int skew_evd_create(skew_evd_handle *h, void *hip_stream)
{
    if (!h) return -1;
    *h = nullptr;
    int rc = check_device();
    if (rc) return rc;
    skew_evd_handle hh = new skew_evd_handle_s();
    hh->stream = (hipStream_t)hip_stream;
    HCHK(hipGetDevice(&hh->device));
    for (int i = 0; i < NSTAGE_EV; ++i) HCHK(hipEventCreate(&hh->ev[i]));
    HCHK(hipHostMalloc((void **)&hh->ctl_host, 64 * sizeof(unsigned), hipHostMallocDefault));
    *h = hh;
    return SKEW_EVD_OK;
}

int skew_evd_destroy(skew_evd_handle h)
{
    if (!h) return -1;
    (void)hipStreamSynchronize(h->stream);
    if (h->ws) (void)hipFree(h->ws);
    for (int i = 0; i < NSTAGE_EV; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    delete h;
    return SKEW_EVD_OK;
}

int skew_evd_ex(skew_evd_handle h, int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr,
                double *Z_im, int ldzi, const skew_evd_opts *opts, skew_evd_info *info)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    if (nev < 0 || nev > (n + 1) / 2) return -5;
    if (nev > 0 && !lambda) return -6;
    if (nev > 0 && !Z_re) return -7;
    if (ldzr < std::max(1, n)) return -8;
    if (nev > 0 && !Z_im) return -9;
    if (ldzi < std::max(1, n)) return -10;
    if (validate_opts(opts)) return -11;
    if (info) memset(info, 0, sizeof(*info));
    if (n == 0 || nev == 0) return SKEW_EVD_OK;
    return solve(h, n, A, lda, nev, lambda, Z_re, ldzr, Z_im, ldzi, opts, info);
}

static skew_evd_handle default_handle(int *rc)
{
    static thread_local skew_evd_handle hd[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *rc = SKEW_EVD_ERR_NODEVICE;
        return nullptr;
    }
    if (!hd[dev]) {
        *rc = skew_evd_create(&hd[dev], nullptr);
        if (*rc) return nullptr;
    }
    *rc = 0;
    return hd[dev];
}

int skew_evd(int n, const double *A, int lda, int nev, double *lambda, double *Z_re, double *Z_im)
{
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max(1, n)) return -3;
    if (nev < 0 || nev > (n + 1) / 2) return -4;
    if (nev > 0 && !lambda) return -5;
    if (nev > 0 && !Z_re) return -6;
    if (nev > 0 && !Z_im) return -7;
    if (n == 0 || nev == 0) return SKEW_EVD_OK;
    int rc = check_device();
    if (rc) return rc;
    skew_evd_handle h = default_handle(&rc);
    if (!h) return rc;
    return skew_evd_ex(h, n, A, lda, nev, lambda, Z_re, n, Z_im, n, nullptr, nullptr);
}

int skew_evd_batched(skew_evd_handle h, int count, const int *n, const double *const *A, const int *lda,
                     const int *nev, double *const *lambda, double *const *Z_re, double *const *Z_im,
                     const skew_evd_opts *opts, skew_evd_info *info, int *status)
{
    if (!h) return -1;
    if (count < 0) return -2;
    if (count > 0 && (!n || !A || !lda || !nev || !lambda || !Z_re || !Z_im || !status)) {
        if (!n) return -3;
        if (!A) return -4;
        if (!lda) return -5;
        if (!nev) return -6;
        if (!lambda) return -7;
        if (!Z_re) return -8;
        if (!Z_im) return -9;
        return -12;
    }
    if (validate_opts(opts)) return -10;
    int first = 0;
    skew_evd_info acc;
    memset(&acc, 0, sizeof(acc));
    for (int i = 0; i < count; ++i) {
        skew_evd_info one;
        int rc = skew_evd_ex(h, n[i], A[i], lda[i], nev[i], lambda[i], Z_re[i], std::max(1, n[i]), Z_im[i],
                             std::max(1, n[i]), opts, &one);
        status[i] = rc;
        if (rc && !first) first = rc;
        acc.ms_total += one.ms_total;
        for (int s = 0; s < 8; ++s) acc.ms_stage[s] += one.ms_stage[s];
        acc.band = one.band;
    }
    acc.workspace_bytes = h->ws_bytes;
    if (info) *info = acc;
    return first;
}

int skew_evd_band_reduce(skew_evd_handle h, int n, const double *A, int lda, int b, double *band, int ldband)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    if (b < 8 || b > 64 || b % 8) return -5;
    if (n > 0 && !band) return -6;
    if (ldband < b + 1) return -7;
    if (n == 0) return SKEW_EVD_OK;
    Plan p = make_plan(n, 0, b, 0);
    Layout L = plan_layout(p);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    HCHK(hipMemsetAsync(ptr<unsigned>(h, L.ctl), 0, sizeof(unsigned) * 64, h->stream));
    HCHK(hipEventRecord(h->ev[0], h->stream));
    rc = stage_band<double>(h, p, L, A, lda, 1);
    if (rc) return rc;
    HCHK(hipMemcpy2DAsync(band, sizeof(double) * ldband, ptr<double>(h, L.ab), sizeof(double) * (2 * b + 1),
                          sizeof(double) * (b + 1), n, hipMemcpyDeviceToDevice, h->stream));
    return finish_status(h, L);
}

int skew_evd_tridiagonalize(skew_evd_handle h, int n, const double *A, int lda, int b, double *alpha)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    if (b != 0 && (b < 8 || b > 64 || b % 8)) return -5;
    if (n > 1 && !alpha) return -6;
    if (n <= 1) return SKEW_EVD_OK;
    Plan p = make_plan(n, 0, b, 0);
    Layout L = plan_layout(p);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    HCHK(hipMemsetAsync(ptr<unsigned>(h, L.ctl), 0, sizeof(unsigned) * 64, h->stream));
    HCHK(hipEventRecord(h->ev[0], h->stream));
    rc = stage_band<double>(h, p, L, A, lda, 1);
    if (rc) return rc;
    rc = stage_chase(h, p, L);
    if (rc) return rc;
    HCHK(hipMemcpyAsync(alpha, ptr<double>(h, L.alpha), sizeof(double) * (n - 1), hipMemcpyDeviceToDevice,
                        h->stream));
    return finish_status(h, L);
}

int skew_evd_tridiag_eig(skew_evd_handle h, int n, const double *alpha, int nev, double *lambda, double *Q, int ldq)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 1 && !alpha) return -3;
    if (nev < 0 || nev > (n + 1) / 2) return -4;
    if (nev > 0 && !lambda) return -5;
    if (nev > 0 && !Q) return -6;
    if (ldq < std::max(1, n)) return -7;
    if (n == 0 || nev == 0) return SKEW_EVD_OK;
    Plan p = make_plan(n, nev, 16, 0);
    p.npanels = 0;
    p.ngroups = 0;
    p.nsig = 0;
    Layout L = plan_layout(p);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    HCHK(hipMemsetAsync(ptr<unsigned>(h, L.ctl), 0, sizeof(unsigned) * 64, h->stream));
    if (n == 1) {
        HCHK(hipMemsetAsync(ptr<double>(h, L.alpha), 0, sizeof(double), h->stream));
        alpha = ptr<double>(h, L.alpha);
    }
    rc = stage_tridiag(h, p, L, alpha, nev, lambda, Q, ldq);
    if (rc) return rc;
    return finish_status(h, L);
}

const char *skew_evd_status_string(int status)
{
    switch (status) {
    case SKEW_EVD_OK: return "success";
    case SKEW_EVD_ERR_NONFINITE: return "non-finite entry in the strict lower triangle of A";
    case SKEW_EVD_ERR_NOCONV: return g_errtext[0] ? g_errtext : "no convergence / device wait gave up";
    case SKEW_EVD_WARN_REFINE: return "refinement stopped above its tolerance";
    case SKEW_EVD_ERR_NOMEM: return g_errtext[0] ? g_errtext : "out of device memory";
    case SKEW_EVD_ERR_HIP: return g_errtext[0] ? g_errtext : "HIP runtime error";
    case SKEW_EVD_ERR_NODEVICE: return "no usable HIP device";
    default: return status < 0 ? "invalid argument" : "unknown status";
    }
}

int skew_evd_version(void) { return 100; }

}  // extern "C"
