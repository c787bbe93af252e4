// C-ABI of the skew-symmetric eigensolver and the host-side stage drivers.
// The host only validates arguments, plans the workspace and enqueues kernels
// on the handle's stream; every arithmetic step runs in the device kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>
#include <algorithm>
#include <chrono>
#include <map>
#include <type_traits>
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
constexpr int SKEW_EVD_REFINE_CLUSTER = 100;   // internal: refinement met unresolvable clusters
constexpr int ORTH_NB = 64;

struct Plan {
    int n = 0, nev = 0, b = 0, nb2 = 0, prec = 0;
    int npanels = 0, ngroups = 0, nsig = 0;
    int orth_window = 0;
    bool hh_panels = false;   // every panel by the Householder kernel (no Cholesky QR)
    bool onestage = false;    // one-stage reduction to tridiagonal form (no band, no chase)
    bool herm = false;        // the complex Hermitian route on iA (one stage, complex reflectors)
};

}  // namespace

struct skew_evd_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ev[NSTAGE_EV] = {};
    unsigned *ctl_host = nullptr;   // pinned copy of the control words
    // per-kernel timing (opts.profile)
    bool prof = false;
    int prof_only = -1;             // >= 0: time only this kernel class
    std::vector<hipEvent_t> kev;
    size_t kev_used = 0;
    struct KRec { int kid; size_t e0, e1; };
    std::vector<KRec> krec;
    size_t kopen[SKEW_EVD_NKERN] = {};
    int refine_passes = 0;
    bool async = false;             // enqueue only: no stage events, no host waits (batched form)
    char *ws2 = nullptr;            // Bethe-Salpeter route: M / L, K, back-transformation
    size_t ws2_bytes = 0;
    bool noalloc = false;           // allocation-free entry point: fixed buffers, no events created
    double *lam_host = nullptr;     // pinned: eigenvalues, ||T||, then the polishing shifts
    size_t lam_cap = 0;
    int polish_lo = 0, polish_hi = 0;   // vectors [lo, hi) get the polishing step
    std::vector<int> win0;          // per Gram-Schmidt block: first vector of its window
    hipEvent_t win_ev = nullptr;    // the eigenvalues' copy to lam_host is complete
    unsigned debug = 0;             // opts.debug of the current call
    // second stream: the T factors of the stage-2 groups run on it beside
    // the tridiagonal solve
    hipStream_t aux = nullptr;
    hipEvent_t aux_ev[4] = {};
    bool merges_started = false;   // this solve queued the stage-1 merges before the chase
    // batched form: sub-streams with an event each, a fork event, and pinned
    // host images of the batched chase's descriptors and the status words
    std::vector<hipStream_t> sub_streams;
    std::vector<hipEvent_t> bev;
    hipEvent_t bev0 = nullptr;
    char *bhost = nullptr;
    size_t bhost_cap = 0;
    // the batch's launches as a HIP graph, captured on bstream for one batch
    // signature (bkey) and replayed while the signature repeats; the
    // generations change whenever the workspace or the pinned descriptors
    // are reallocated (an address can be reused)
    hipStream_t bstream = nullptr;
    hipEvent_t bgev[2] = {};
    hipGraphExec_t bgraph = nullptr;
    std::vector<uintptr_t> bkey;
    unsigned long ws_gen = 0, bhost_gen = 0;
    // band-width autotuner: (precision, size class) -> (band, best wall ms)
    struct Tuned {
        int band, panel;
        double ms;
    };
    std::map<int, Tuned> tune;
};

namespace {

// ---------------------------------------------------------------------------
// Workspace layout.  Offsets are 256-byte aligned.
struct Layout {
    size_t W, Vall, Tall, tauall, Ypart, Y0, Wd, Gp, Tx, part, ab, goff, V2, tau2, T2, V2t, alpha, a2, stats,
        lam, gcnt, U0, U1, U2, Lm, Sw, Yiv, ivfac, pshift, Qd, Z, Wos, oss, Wim, Vim, Tim, tauc, Wosi, dgl, Wp2, cq, cqGp, Wp, Wt2, Pp, P, Gp2, Rinv, Tmp, ctl, rX, rXn, rP, rS, rG, rE, rlam,
        rstat, Tm, total;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// offset (elements) of panel j's V_j in Vall: sum over i < j of (n - (i+1) b) b
// (two-stage), of (n - i b - 1) b (one-stage: panel i's reflectors start at row
// i b + 1)
size_t voff(const Plan &p, int j)
{
    const size_t n = p.n, b = p.b, jj = j;
    if (p.onestage) return b * (jj * (n - 1) - b * jj * (jj - 1) / 2);
    return b * (jj * n - b * jj * (jj + 1) / 2);
}

int tn_parts_max() { return 32; }

// Row splits of the Gram products of the Cholesky-QR panel path: about 128
// rows per workgroup (a short chain of K-chunks), at most cholqr_max_splits().
int cholqr_max_splits() { return 128; }
int cholqr_splits(int m)
{
    int S = (m + 127) / 128;
    return S < 1 ? 1 : (S > cholqr_max_splits() ? cholqr_max_splits() : S);
}

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
    size_t vtot = 0;
    for (int j = 0; j < p.npanels; ++j) vtot += (p.onestage ? n - (size_t)j * b - 1 : n - (size_t)(j + 1) * b) * b;
    L.Vall = take(es * vtot);
    L.Tall = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * b * b);
    L.Tm = take(sizeof(double) * (size_t)(p.npanels / 2 + 1) * 4 * b * b);
    L.tauall = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * b);
    const size_t m0 = n > b ? n - b : 1;
    L.Ypart = take(es * 16 * m0 * b);
    L.Y0 = take(es * m0 * b);
    L.Wd = take(es * m0 * b);
    L.Gp = take(sizeof(double) * (m0 / skew::gram_chunk_rows() + 2) * b * b);
    L.Tx = take(es * 2 * b * b);
    L.part = take(sizeof(double) * skew::panel_qr_part_doubles((int)m0, (int)b));
    L.ab = take(sizeof(double) * (2 * b + 1) * n);
    L.goff = take(sizeof(int) * (p.nsig + 2));
    L.V2 = take(sizeof(double) * (size_t)p.ngroups * b * nb2);
    L.tau2 = take(sizeof(double) * (size_t)p.ngroups * nb2);
    L.T2 = take(sizeof(double) * (size_t)p.ngroups * nb2 * nb2);
    L.V2t = p.prec ? take(es * (size_t)p.ngroups * b * nb2) : 0;
    L.alpha = take(sizeof(double) * n);
    L.a2 = take(sizeof(double) * n);
    L.stats = take(sizeof(double) * 4);
    L.lam = take(sizeof(double) * nev);
    L.gcnt = take(sizeof(int) * (size_t)skew::tri_grid_points((int)nev));
    L.U0 = take(sizeof(double) * n * nev);
    L.U1 = take(sizeof(double) * n * nev);
    L.U2 = take(sizeof(double) * n * nev);
    L.Lm = take(sizeof(double) * n * nev);
    L.Sw = take(n * nev);
    L.Yiv = take(sizeof(double) * n * nev);
    L.ivfac = take(sizeof(double) * 2 * nev);
    L.pshift = take(sizeof(double) * nev);
    L.Qd = take(sizeof(double) * n * nev);
    L.Z = take(es * n * 2 * nev);
    L.cq = take(sizeof(double) * skew::cholqr_scratch_doubles());
    L.cqGp = take(sizeof(double) * (size_t)cholqr_max_splits() * b * b);
    L.Wp = take(sizeof(double) * tn_parts_max() * b * 2 * nev);
    L.Wt2 = take(sizeof(double) * 2 * b * 2 * nev);
    // a window covers at least orth_window earlier vectors and grows to every
    // earlier vector of a cluster (up to nev)
    const size_t wmax = std::max((size_t)p.nev, (size_t)ORTH_NB);
    L.Pp = take(sizeof(double) * tn_parts_max() * wmax * ORTH_NB);
    L.P = take(sizeof(double) * wmax * ORTH_NB);
    L.Gp2 = take(sizeof(double) * std::max(tn_parts_max(), cholqr_max_splits()) * ORTH_NB * ORTH_NB);
    L.Rinv = take(sizeof(double) * ORTH_NB * ORTH_NB);
    L.Tmp = take(sizeof(double) * n * ORTH_NB);
    L.ctl = take(sizeof(unsigned) * (64 + n));
    L.Wos = p.onestage ? take(sizeof(double) * n * 64) : 0;
    L.oss = p.onestage ? take(sizeof(double) * (p.herm ? skew::herm_scratch_doubles((int)n)
                                                         : skew::onestage_scratch_doubles((int)n)))
                       : 0;
    L.Wim = L.Vim = L.Tim = L.tauc = L.Wosi = L.dgl = L.Wp2 = 0;
    if (p.herm) {
        // the imaginary planes of H, V, T and W, complex tau, the diagonal,
        // and the second set of GEMM partials of the back-transformation
        L.Wim = take(sizeof(double) * n * n);
        L.Vim = take(sizeof(double) * vtot);
        L.Tim = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * b * b);
        L.tauc = take(sizeof(double) * (size_t)std::max(p.npanels, 1) * 2 * b);
        L.Wosi = take(sizeof(double) * n * 64);
        L.dgl = take(sizeof(double) * n);
        L.Wp2 = take(sizeof(double) * tn_parts_max() * b * 2 * nev);
    }
    if (p.prec) {
        const size_t ncx = n;   // 2 nev columns (2 nev - 1 for odd n); nev = ceil(n/2) for the full half
        const size_t nc = std::max((size_t)2 * nev, ncx);
        L.rX = take(sizeof(double) * n * nc);
        L.rXn = take(sizeof(double) * n * nc);
        L.rP = take(sizeof(double) * n * nc);
        L.rS = take(sizeof(double) * nc * nc);
        L.rG = take(sizeof(double) * nc * nc);
        L.rE = take(sizeof(float) * nc * nc);
        L.rlam = take(sizeof(double) * (nev + 1));
        L.rstat = take(sizeof(double) * 8);
    } else {
        L.rX = L.rXn = L.rP = L.rS = L.rG = L.rE = L.rlam = L.rstat = 0;
    }
    L.total = off;
    return L;
}

// control words
enum { CTL_FLAGS = 0, CTL_ERR = 1, CTL_BAR = 2, CTL_QRFLAG = 3, CTL_PROGRESS = 64 };

// Fixed band rule (opts.band = 0 without the autotuner).  The autotuner
// picks 64 for every size class from 128 to 1024 on gfx950: the wider panels'
// MFMA efficiency outweighs the longer bulge chase there too.
int auto_band(int n)
{
    if (n >= 128) return 64;
    return 16;
}

// Fixed panel rule (opts.panel_method = 0 without the autotuner): Cholesky QR
// everywhere.  (Householder panels for every order up to 1024 made the batch
// of 512 uneven problems slower, 1.76 s against 1.19 s: the autotuner picks
// them per size class only where they win.)
constexpr int HH_PANEL_NMAX = 0;

// Fixed part of the Gram-Schmidt windows (beyond it a window extends over a
// cluster, see plan_windows): up to 2048 vectors every vector, else the 256
// before the block.  Inverse iteration leaves a component of size about
// eps ||T|| / gap along the vector of an eigenvalue a gap away; 256 vectors
// span about 256 / nev of the spectrum (gaps of several percent of ||T|| for
// spread spectra), so the components left behind sum to orders of magnitude
// below the orthogonality tolerance, and closer eigenvalues are covered by
// the cluster rule.
int orth_window_for(int nev) { return nev <= 2048 ? nev : 256; }

Plan make_plan(int n, int nev, int b, int prec, int panel = SKEW_EVD_PANEL_AUTO, bool onestage = false,
               bool herm = false)
{
    Plan p;
    if (onestage || herm) {
        // panels of 64 columns over columns 0 .. n-2 (the last one with a sub-diagonal entry)
        p.onestage = true;
        p.herm = herm;
        p.n = n;
        p.nev = nev;
        p.b = p.nb2 = 64;
        p.npanels = n >= 2 ? (n - 1 + 63) / 64 : 0;
        p.orth_window = orth_window_for(nev);
        return p;
    }
    p.hh_panels = panel == SKEW_EVD_PANEL_HOUSEHOLDER || (panel == SKEW_EVD_PANEL_AUTO && n <= HH_PANEL_NMAX);
    p.n = n;
    p.nev = nev;
    p.prec = prec;
    p.b = b > 0 ? b : auto_band(n);
    p.nb2 = p.b;
    p.npanels = 0;
    for (int c0 = 0; c0 + p.b < n - 1; c0 += p.b) ++p.npanels;
    p.nsig = n > 2 ? (n - 2 + p.nb2 - 1) / p.nb2 : 0;
    p.ngroups = skew::chase_ngroups(n, p.b, p.nb2, nullptr);
    p.orth_window = orth_window_for(nev);
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
        if (h->aux) HCHK(hipStreamSynchronize(h->aux));
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
    ++h->ws_gen;
    return SKEW_EVD_OK;
}

template <typename T> T *ptr(skew_evd_handle h, size_t off) { return (T *)(h->ws + off); }

// stage event i on the handle's stream (none in the enqueue-only mode)
hipError_t ev_record(skew_evd_handle h, int i)
{
    if (h->async || !h->ev[i]) return hipSuccess;
    return hipEventRecord(h->ev[i], h->stream);
}

// Kernel timers: an event before and after the launches of a main kernel.
hipError_t kt_event(skew_evd_handle h, size_t *idx)
{
    if (h->kev_used == h->kev.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        h->kev.push_back(e);
    }
    *idx = h->kev_used++;
    return hipEventRecord(h->kev[*idx], h->stream);
}
hipError_t kt_begin(skew_evd_handle h, int kid)
{
    if (!h->prof || (h->prof_only >= 0 && kid != h->prof_only)) return hipSuccess;
    return kt_event(h, &h->kopen[kid]);
}
hipError_t kt_end(skew_evd_handle h, int kid)
{
    if (!h->prof || (h->prof_only >= 0 && kid != h->prof_only)) return hipSuccess;
    size_t e1;
    hipError_t r = kt_event(h, &e1);
    h->krec.push_back({kid, h->kopen[kid], e1});
    return r;
}
void kt_reset(skew_evd_handle h, bool on, int only = -1)
{
    h->prof = on;
    h->prof_only = only;
    h->kev_used = 0;
    h->krec.clear();
}
// after synchronisation
void kt_collect(skew_evd_handle h, skew_evd_info *info)
{
    if (!info || !h->prof) return;
    for (const auto &r : h->krec) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->kev[r.e0], h->kev[r.e1]) == hipSuccess) {
            info->kern[r.kid].ms += ms;
            info->kern[r.kid].launches += 1;
        }
    }
}

// Algorithmic flop and byte counts of the main kernels for a plan.
void kt_counts(const struct Plan &p, skew_evd_info *info)
{
    if (!info) return;
    const double n = p.n, nev = p.nev, b = p.b, es = p.prec ? 4.0 : 8.0;
    double sm = 0.0, sm2 = 0.0;
    for (int j = 0; j < p.npanels; ++j) {
        double m = n - (double)(j + 1) * b;
        sm += m;
        sm2 += m * m;
    }
    skew_evd_kstat *k = info->kern;
    k[SKEW_EVD_K_PANEL].flops = 2.0 * sm * b * b;
    k[SKEW_EVD_K_PANEL].bytes = 2.0 * es * sm * b;
    k[SKEW_EVD_K_PANEL].bound = SKEW_EVD_BOUND_ALU;
    k[SKEW_EVD_K_SYMM].flops = 2.0 * sm2 * b + 6.0 * sm * b * b;
    k[SKEW_EVD_K_SYMM].bytes = es * sm2 / 2.0;
    k[SKEW_EVD_K_SYMM].bound = SKEW_EVD_BOUND_MFMA;
    k[SKEW_EVD_K_SYR2K].flops = 2.0 * sm2 * b;
    k[SKEW_EVD_K_SYR2K].bytes = es * sm2;
    k[SKEW_EVD_K_SYR2K].bound = SKEW_EVD_BOUND_MFMA;
    k[SKEW_EVD_K_CHASE].flops = 6.0 * n * n * b;
    k[SKEW_EVD_K_CHASE].bytes = 8.0 * (2.0 * b + 1.0) * n * 2.0 + 8.0 * n * n / 2.0;
    k[SKEW_EVD_K_CHASE].bound = SKEW_EVD_BOUND_ALU;
    k[SKEW_EVD_K_TRIDIAG].flops = 3.0 * 14.0 * 16.0 * n * nev + 4.0 * n * nev * p.orth_window;
    k[SKEW_EVD_K_TRIDIAG].bytes = 8.0 * n * nev * 8.0;
    k[SKEW_EVD_K_TRIDIAG].bound = SKEW_EVD_BOUND_ALU;
    k[SKEW_EVD_K_BT2].flops = 4.0 * n * n * nev;
    k[SKEW_EVD_K_BT2].bytes = es * (2.0 * 2.0 * n * nev + n * n / 2.0);
    k[SKEW_EVD_K_BT2].bound = SKEW_EVD_BOUND_MFMA;
    k[SKEW_EVD_K_BT1].flops = 8.0 * b * nev * sm;
    k[SKEW_EVD_K_BT1].bytes = es * 3.0 * sm * 2.0 * nev;
    k[SKEW_EVD_K_BT1].bound = SKEW_EVD_BOUND_MFMA;
    k[SKEW_EVD_K_REFINE].bound = SKEW_EVD_BOUND_MFMA;
    if (p.onestage) {
        // the panel loop is the whole reduction: per column, the skew matrix-
        // vector product streams the stored trailing triangle (m_c^2 / 2
        // words, 2 m_c^2 flops); per panel, the rank-2b update reads and
        // writes it (M^2 words, 2 M^2 b flops)
        double sc = 0.0, sp = 0.0, sb = 0.0;
        for (int c = 0; c + 1 < p.n; ++c) {
            const double m = n - c - 1.0;
            sc += m * m;
        }
        for (int j = 0; j < p.npanels; ++j) {
            const double M = n - (double)(j + 1) * b;
            if (M > 1.0) sp += M * M;
            sb += n - (double)j * b - 1.0;
        }
        for (int q = SKEW_EVD_K_SYMM; q <= SKEW_EVD_K_BT2; ++q)
            if (q != SKEW_EVD_K_TRIDIAG) k[q].flops = k[q].bytes = 0.0;
        // complex Hermitian route: entries of 16 bytes, 8 flops per complex
        // multiply-add, twice the real back-transformation's products
        const double cw = p.herm ? 2.0 : 1.0, cf = p.herm ? 4.0 : 1.0;
        k[SKEW_EVD_K_PANEL].flops = cf * (2.0 * sc + 2.0 * sp * b);
        k[SKEW_EVD_K_PANEL].bytes = cw * 8.0 * (sc / 2.0 + sp);
        k[SKEW_EVD_K_PANEL].bound = SKEW_EVD_BOUND_HBM;
        k[SKEW_EVD_K_BT1].flops = cw * 8.0 * b * nev * sb;
        k[SKEW_EVD_K_BT1].bytes = cw * 8.0 * 3.0 * sb * 2.0 * nev;
    }
}

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
    (void)check_finite;   // the non-finite flag is read when the call completes
    HCHK(ev_record(h, 1));
    unsigned bar_base = 0;
    for (int j = 0; j < p.npanels; ++j) {
        const int c0 = j * b, r0 = c0 + b, m = n - r0;
        T *Vd = ptr<T>(h, L.Vall) + voff(p, j);
        double *Tf = ptr<double>(h, L.Tall) + (size_t)j * b * b;
        double *tauj = ptr<double>(h, L.tauall) + (size_t)j * b;
        HCHK(kt_begin(h, SKEW_EVD_K_PANEL));
        const unsigned *skip = nullptr;
        if (m >= b && !p.hh_panels) {
            // Cholesky QR twice + Householder reconstruction (Gram matrices
            // and the small factorizations in FP64 also in the FP32 form); the
            // Householder panel kernel below runs only when this path flags
            // the panel
            T *P = W + (size_t)c0 * n + r0;
            T *Vq = Vd;
            double *cq = ptr<double>(h, L.cq), *Gq = ptr<double>(h, L.cqGp);
            unsigned *qf = ctl + CTL_QRFLAG;
            const size_t BB = (size_t)64 * 64;
            // the Gram matrices (the reflectors' norms) are formed in FP64 in both forms
            auto gram = [&](const T *X, int ldx) -> int {
                if constexpr (std::is_same<T, float>::value)
                    return skew::launch_gemm_tn_part_f64(X, ldx, X, ldx, b, b, m, Gq, st, cholqr_splits(m));
                else
                    return skew::launch_gemm_tn_part<T>(X, ldx, X, ldx, b, b, m, Gq, st, cholqr_splits(m));
            };
            // few partials are summed by the Cholesky kernel itself, many by
            // a parallel reduction first (the same order of summation)
            auto chol = [&](int S, int pass) {
                if (S <= 16) {
                    skew::launch_chol_qr(b, pass, cq, qf, st, Gq, S);
                } else {
                    skew::launch_gram_reduce(Gq, S, b * b, cq + skew::CQ_G * BB, st);
                    skew::launch_chol_qr(b, pass, cq, qf, st);
                }
            };
            chol(gram(P, n), 1);
            skew::launch_gemm_nn<T>(P, n, cq + skew::CQ_R1INV * BB, 1, m, b, b, Vq, m, 1.0, 0, st);
            chol(gram(Vq, m), 2);
            skew::launch_gemm_nn<T>(Vq, m, cq + skew::CQ_R2INV * BB, 1, m, b, b, Vq, m, 1.0, 0, st);
            skew::launch_hh_rebuild<T>(Vq, m, b, P, n, cq, Tf, tauj, qf, st);
            if (m > b)
                skew::launch_gemm_nn<T>(Vq + b, m, cq + skew::CQ_UINV * BB, 1, m - b, b, b, Vq + b, m, 1.0, 0, st);
            skip = qf;
        }
        HCHK(skew::launch_panel_qr<T>(W, n, c0, r0, m, b, Vd, tauj, Tf, ptr<double>(h, L.part), ctl + CTL_BAR,
                                      bar_base, ctl + CTL_ERR, skip, st));
        HCHK(kt_end(h, SKEW_EVD_K_PANEL));
        bar_base += (unsigned)((std::min(m, b) + 1) * skew::panel_qr_groups(m));
        if (m > 1) {
            HCHK(kt_begin(h, SKEW_EVD_K_SYMM));
            skew::launch_stage1_w<T>(W, n, r0, m, b, Vd, Tf, ptr<T>(h, L.Ypart), ptr<T>(h, L.Y0), ptr<T>(h, L.Wd),
                                     ptr<double>(h, L.Gp), ptr<T>(h, L.Tx), st);
            HCHK(kt_end(h, SKEW_EVD_K_SYMM));
            HCHK(kt_begin(h, SKEW_EVD_K_SYR2K));
            skew::launch_stage1_syr2k<T>(W, n, r0, m, b, Vd, ptr<T>(h, L.Wd), st);
            HCHK(kt_end(h, SKEW_EVD_K_SYR2K));
        }
        HCHK(hipGetLastError());
    }
    skew::launch_band_extract<T>(W, n, n, b, ptr<double>(h, L.ab), 2 * b + 1, st);
    HCHK(hipGetLastError());
    HCHK(ev_record(h, 2));
    return SKEW_EVD_OK;
}

// Everything the chase needs besides the band: the group offsets of its
// reflectors (device-side), zeroed reflector storage, counters and ticket.
void chase_prepare(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, b = p.b;
    skew::launch_goff(n, b, p.nb2, ptr<int>(h, L.goff), st);
    if (p.ngroups > 0) {
        skew::launch_fill32(ptr<double>(h, L.V2), 0u, 2 * (size_t)p.ngroups * b * p.nb2, st);
        skew::launch_fill32(ptr<double>(h, L.tau2), 0u, 2 * (size_t)p.ngroups * p.nb2, st);
    }
    skew::launch_fill32(ptr<unsigned>(h, L.ctl) + CTL_PROGRESS, 0u, (size_t)n, st);   // counters and the ticket
}

int stage_chase(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, b = p.b;
    chase_prepare(h, p, L);
    unsigned *ctl = ptr<unsigned>(h, L.ctl);
    HCHK(kt_begin(h, SKEW_EVD_K_CHASE));
    HCHK(skew::launch_chase(ptr<double>(h, L.ab), 2 * b + 1, n, b, p.nb2, ptr<double>(h, L.V2),
                            ptr<double>(h, L.tau2), ptr<int>(h, L.goff), ctl + CTL_PROGRESS, ctl + CTL_ERR,
                            ptr<double>(h, L.alpha), st));
    HCHK(kt_end(h, SKEW_EVD_K_CHASE));
    HCHK(ev_record(h, 3));
    return SKEW_EVD_OK;
}

// Gram-Schmidt windows.  Inverse iteration gives vectors accurate to about
// eps ||T|| / gap, so vectors of eigenvalues closer than a fraction of ||T||
// must be orthogonalized against each other.  The window of the block that
// starts at vector b0 covers the orth_window vectors before it and, beyond
// them, every earlier vector whose eigenvalue lies within 1e-3 ||T|| of
// lambda_b0 (the cluster criterion of LAPACK's dstein), so a cluster of any
// width is orthogonalized as a whole.
//
// Degenerate clusters (consecutive eigenvalues closer than DEGEN_TOL ||T||,
// numerically equal) need one more step.  Their inverse-iteration vectors are
// random within the invariant subspace, so the last blocks of a cluster that
// fills its subspace are ill-conditioned, and orthonormalizing them magnifies
// the small components outside the subspace (residual and orthogonality
// errors up to ~1e-9 for clusters of 2048).  After the Gram-Schmidt pass each
// such vector gets one inverse-iteration step with the shift lambda_c0 - d
// (lambda_c0 the cluster's smallest value, d = max(1e-10 ||T||, 1e3 x the
// cluster's width)): every direction inside the cluster is magnified by
// nearly the same 1/d, so the basis stays well-conditioned, while the
// components outside shrink by d / gap.  A second Gram-Schmidt pass from the
// first polished block then restores orthonormality.
constexpr double ORTH_CLUSTER = 1e-3;
constexpr double DEGEN_TOL = 1e3 * 2.220446049250313e-16;

bool windows_fixed(const Plan &p, int nev) { return nev <= p.orth_window; }

// enqueue the copy of the eigenvalues and ||T|| to the host (after the bisection)
int fetch_windows(skew_evd_handle h, const Plan &p, const Layout &L, const double *lam_dev, int nev)
{
    (void)p;
    if (h->async) return SKEW_EVD_OK;
    if (!h->win_ev && !h->noalloc) HCHK(hipEventCreateWithFlags(&h->win_ev, hipEventDisableTiming));
    if ((size_t)2 * nev + 1 > h->lam_cap) {
        if (h->noalloc) {
            snprintf(g_errtext, sizeof(g_errtext), "eigenvalue buffer of the allocation-free path too small");
            return SKEW_EVD_ERR_NOMEM;
        }
        if (h->lam_host) HCHK(hipHostFree(h->lam_host));
        h->lam_host = nullptr;
        h->lam_cap = 0;
        HCHK(hipHostMalloc((void **)&h->lam_host, sizeof(double) * (2 * nev + 1), hipHostMallocDefault));
        h->lam_cap = 2 * nev + 1;
    }
    HCHK(hipMemcpyAsync(h->lam_host, lam_dev, sizeof(double) * nev, hipMemcpyDeviceToHost, h->stream));
    HCHK(hipMemcpyAsync(h->lam_host + nev, ptr<double>(h, L.stats), sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
    if (h->win_ev) HCHK(hipEventRecord(h->win_ev, h->stream));
    return SKEW_EVD_OK;
}

// wait for that copy (work queued after it keeps running), set the windows,
// and find the degenerate clusters with their polishing shifts
int plan_windows(skew_evd_handle h, const Plan &p, int nev)
{
    h->win0.clear();
    h->polish_lo = h->polish_hi = 0;
    if (h->async) return SKEW_EVD_OK;       // fixed windows; degenerate clusters are flagged on the device
    if (h->win_ev) HCHK(hipEventSynchronize(h->win_ev));
    else HCHK(hipStreamSynchronize(h->stream));
    const double *lam = h->lam_host;
    const double g = h->lam_host[nev];      // ||T||_inf
    if (!windows_fixed(p, nev)) {
        const int nblk = (nev + ORTH_NB - 1) / ORTH_NB;
        const double tau = ORTH_CLUSTER * g;
        for (int k = 0; k < nblk; ++k) {
            const int b0 = k * ORTH_NB;
            const int wfix = std::max(0, b0 - p.orth_window);
            const int wclu = (int)(std::lower_bound(lam, lam + b0, lam[b0] - tau) - lam);
            h->win0.push_back(std::min(wfix, wclu));
        }
    }
    double *sh = h->lam_host + nev + 1;
    int lo = -1, hi = -1;
    for (int k = 0; k < nev;) {
        int j = k;
        while (j + 1 < nev && lam[j + 1] - lam[j] <= DEGEN_TOL * g) ++j;
        if (j > k && g > 0.0) {
            const double d = std::max(1e-10 * g, 1e3 * (lam[j] - lam[k]));
            for (int c = k; c <= j; ++c) sh[c] = lam[k] - d;
            if (lo < 0) lo = k;
            hi = j + 1;
        } else {
            sh[k] = lam[k];
        }
        k = j + 1;
    }
    if (lo >= 0) {
        h->polish_lo = lo;
        h->polish_hi = hi;
    }
    return SKEW_EVD_OK;
}

// Block Gram-Schmidt in eigenvalue order (window of earlier vectors, then a
// Cholesky-QR of the block).  A window that a cluster extends beyond the
// fixed length is projected out twice (classical Gram-Schmidt needs the
// second pass when a block is nearly in the span of its window).
int orthogonalize(skew_evd_handle h, const Plan &p, const Layout &L, double *Q, int ldq, int n, int nev,
                  int first = 0)
{
    hipStream_t st = h->stream;
    for (int b0 = first; b0 < nev; b0 += ORTH_NB) {
        const int nb = std::min(ORTH_NB, nev - b0);
        const int w0 = h->win0.empty() ? std::max(0, b0 - p.orth_window) : h->win0[b0 / ORTH_NB];
        const int wl = b0 - w0;
        const int passes = wl > p.orth_window ? 2 : 1;
        double *Qb = Q + (size_t)b0 * ldq;
        for (int pass = 0; wl > 0 && pass < passes; ++pass) {
            const double *Qw = Q + (size_t)w0 * ldq;
            // short windows: 128-row chunks (a short chain of K-chunks per
            // workgroup) as far as the partials' buffer holds them
            const size_t wmax = std::max((size_t)p.nev, (size_t)ORTH_NB);
            const int S_req = std::min({128, (int)((size_t)tn_parts_max() * wmax / (size_t)wl), (n + 127) / 128});
            int S = skew::launch_gemm_tn_part<double>(Qw, ldq, Qb, ldq, wl, nb, n, ptr<double>(h, L.Pp), st,
                                                      S_req > tn_parts_max() ? S_req : 0);
            skew::launch_gram_reduce(ptr<double>(h, L.Pp), S, wl * nb, ptr<double>(h, L.P), st);
            skew::launch_gemm_nn<double>(Qw, ldq, ptr<double>(h, L.P), 1, n, nb, wl, Qb, ldq, -1.0, 1, st);
        }
        // the block's Gram matrix: short row chunks (a short chain of K-chunks
        // per workgroup), their partials summed in parallel (into P, free here)
        int S = skew::launch_gemm_tn_part<double>(Qb, ldq, Qb, ldq, nb, nb, n, ptr<double>(h, L.Gp2), st,
                                                  cholqr_splits(n));
        skew::launch_gram_reduce(ptr<double>(h, L.Gp2), S, nb * nb, ptr<double>(h, L.P), st);
        skew::launch_chol_inv(ptr<double>(h, L.P), 1, nb, ptr<double>(h, L.Rinv), st);
        skew::launch_gemm_nn<double>(Qb, ldq, ptr<double>(h, L.Rinv), 1, n, nb, nb, ptr<double>(h, L.Tmp), n, 1.0, 0,
                                     st);
        skew::launch_copy_cols<double>(ptr<double>(h, L.Tmp), n, Qb, ldq, n, nb, st);
        HCHK(hipGetLastError());
    }
    return SKEW_EVD_OK;
}

int start_bt2_factors(skew_evd_handle h, const Plan &p, const Layout &L, bool merges_started);

// One-stage reduction (Section 2.3.1): the strict lower triangle into W, then
// the panels of 64 columns; alpha, the panels' V and T (kept for the
// back-transformation) and tau.  The chase's stage events mark no time.
int stage_onestage(skew_evd_handle h, const Plan &p, const Layout &L, const double *A, int lda)
{
    hipStream_t st = h->stream;
    const int n = p.n;
    double *W = ptr<double>(h, L.W);
    skew::launch_ingest<double>(A, lda, n, W, n, ptr<unsigned>(h, L.ctl) + CTL_FLAGS, st);
    HCHK(hipGetLastError());
    HCHK(ev_record(h, 1));
    HCHK(kt_begin(h, SKEW_EVD_K_PANEL));
    for (int j = 0; j < p.npanels; ++j) {
        const int c0 = 64 * j, nb = std::min(64, n - 1 - c0), ldv = n - c0 - 1;
        double *Vp = ptr<double>(h, L.Vall) + voff(p, j);
        double *Tp = ptr<double>(h, L.Tall) + (size_t)j * 64 * 64;
        if (nb < 64) {                      // the last panel: unused reflectors are zero
            skew::launch_fill32(Vp + (size_t)nb * ldv, 0u, 2 * (size_t)(64 - nb) * ldv, st);
            skew::launch_fill32(Tp, 0u, 2 * 64 * 64, st);
        }
        skew::launch_onestage_panel(W, n, n, c0, nb, Vp, ptr<double>(h, L.Wos), ldv,
                                    ptr<double>(h, L.tauall) + (size_t)j * 64, Tp, ptr<double>(h, L.alpha),
                                    ptr<double>(h, L.oss), st);
        HCHK(hipGetLastError());
    }
    HCHK(kt_end(h, SKEW_EVD_K_PANEL));
    HCHK(ev_record(h, 2));
    HCHK(ev_record(h, 3));
    return SKEW_EVD_OK;
}

// Its back-transformation: D, then Z <- (I - V_j T_j V_j^T) Z for the panels in
// reverse (rows from 64 j + 1).
int stage_bt_onestage(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, nev = p.nev;
    double *Z = ptr<double>(h, L.Z);
    skew::launch_dscale<double>(ptr<double>(h, L.Qd), n, n, nev, Z, n, st);
    HCHK(ev_record(h, 5));
    HCHK(kt_begin(h, SKEW_EVD_K_BT1));
    for (int j = p.npanels - 1; j >= 0; --j) {
        const int c0 = 64 * j, m = n - c0 - 1;
        skew::launch_bt1_block<double>(Z, n, c0 + 1, m, 2 * nev, ptr<double>(h, L.Vall) + voff(p, j), 64, nullptr,
                                       0, ptr<double>(h, L.Tall) + (size_t)j * 64 * 64, 64, ptr<double>(h, L.Wp),
                                       ptr<double>(h, L.Wt2), st);
        HCHK(hipGetLastError());
    }
    HCHK(kt_end(h, SKEW_EVD_K_BT1));
    HCHK(ev_record(h, 6));
    return SKEW_EVD_OK;
}

// The complex Hermitian route on H = iA: the lower triangle of H as two
// planes (real part 0, imaginary part the strict lower triangle of A), then
// the panels of 64 columns; the real tridiagonal matrix (diagonal dgl,
// off-diagonal alpha), the panels' complex V and T kept for the
// back-transformation.
int stage_herm(skew_evd_handle h, const Plan &p, const Layout &L, const double *A, int lda)
{
    hipStream_t st = h->stream;
    const int n = p.n;
    double *Hr = ptr<double>(h, L.W), *Hi = ptr<double>(h, L.Wim);
    skew::launch_fill32(Hr, 0u, 2 * (size_t)n * n, st);
    skew::launch_ingest<double>(A, lda, n, Hi, n, ptr<unsigned>(h, L.ctl) + CTL_FLAGS, st);
    HCHK(hipGetLastError());
    HCHK(ev_record(h, 1));
    HCHK(kt_begin(h, SKEW_EVD_K_PANEL));
    double *d = ptr<double>(h, L.dgl);
    for (int j = 0; j < p.npanels; ++j) {
        const int c0 = 64 * j, nb = std::min(64, n - 1 - c0), ldv = n - c0 - 1;
        double *Vr = ptr<double>(h, L.Vall) + voff(p, j), *Vi = ptr<double>(h, L.Vim) + voff(p, j);
        double *Tr = ptr<double>(h, L.Tall) + (size_t)j * 64 * 64, *Ti = ptr<double>(h, L.Tim) + (size_t)j * 64 * 64;
        if (nb < 64) {                      // the last panel: unused reflectors are zero
            skew::launch_fill32(Vr + (size_t)nb * ldv, 0u, 2 * (size_t)(64 - nb) * ldv, st);
            skew::launch_fill32(Vi + (size_t)nb * ldv, 0u, 2 * (size_t)(64 - nb) * ldv, st);
            skew::launch_fill32(Tr, 0u, 2 * 64 * 64, st);
            skew::launch_fill32(Ti, 0u, 2 * 64 * 64, st);
        }
        skew::launch_herm_panel(Hr, Hi, n, n, c0, nb, Vr, Vi, ptr<double>(h, L.Wos), ptr<double>(h, L.Wosi), ldv,
                                ptr<double>(h, L.tauc) + (size_t)j * 128, Tr, Ti, d, ptr<double>(h, L.alpha),
                                ptr<double>(h, L.oss), st);
        HCHK(hipGetLastError());
    }
    // the last diagonal entry, after the last panel's trailing update
    if (n >= 1)
        HCHK(hipMemcpyAsync(d + (n - 1), Hr + (size_t)(n - 1) * n + (n - 1), sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    HCHK(kt_end(h, SKEW_EVD_K_PANEL));
    HCHK(ev_record(h, 2));
    HCHK(ev_record(h, 3));
    return SKEW_EVD_OK;
}

// Its back-transformation: Z = [S, 0] (S the tridiagonal eigenvectors), then
// Z <- (I - V_j T_j V_j^H) Z for the panels in reverse (rows from 64 j + 1),
// then z = conj(x): the imaginary half negated.
int stage_bt_herm(skew_evd_handle h, const Plan &p, const Layout &L)
{
    hipStream_t st = h->stream;
    const int n = p.n, nev = p.nev;
    double *Z = ptr<double>(h, L.Z);
    skew::launch_copy_cols<double>(ptr<double>(h, L.Qd), n, Z, n, n, nev, st);
    skew::launch_fill32(Z + (size_t)nev * n, 0u, 2 * (size_t)nev * n, st);
    HCHK(ev_record(h, 5));
    HCHK(kt_begin(h, SKEW_EVD_K_BT1));
    for (int j = p.npanels - 1; j >= 0; --j) {
        const int c0 = 64 * j, m = n - c0 - 1;
        skew::launch_herm_bt(Z, n, c0 + 1, m, nev, ptr<double>(h, L.Vall) + voff(p, j),
                             ptr<double>(h, L.Vim) + voff(p, j), ptr<double>(h, L.Tall) + (size_t)j * 64 * 64,
                             ptr<double>(h, L.Tim) + (size_t)j * 64 * 64, ptr<double>(h, L.Wp),
                             ptr<double>(h, L.Wp2), ptr<double>(h, L.Wt2), st);
        HCHK(hipGetLastError());
    }
    skew::launch_negate(Z + (size_t)nev * n, (size_t)nev * n, st);
    HCHK(kt_end(h, SKEW_EVD_K_BT1));
    HCHK(ev_record(h, 6));
    return SKEW_EVD_OK;
}

// Inverse iteration: a vector whose residual exceeds this multiple of ||T||
// is reported as not converged.
constexpr double INVIT_CTOL = 1e-12;

int tridiag_finish(skew_evd_handle h, const Plan &p, const Layout &L, const double *alpha, int nev, double *lam,
                   double *Q, int ldq, const double *diag);

// early_t: start the T factors of the stage-2 groups on the second stream
// once the bisection (which fills the device) is queued, so that they run
// beside the inverse iteration.
int stage_tridiag(skew_evd_handle h, const Plan &p, const Layout &L, const double *alpha, int nev, double *lam,
                  double *Q, int ldq, bool early_t = false, const double *diag = nullptr)
{
    hipStream_t st = h->stream;
    const int n = p.n;
    HCHK(kt_begin(h, SKEW_EVD_K_TRIDIAG));
    skew::launch_tridiag_eigvals(alpha, n, n / 2, nev, ptr<double>(h, L.a2), ptr<double>(h, L.stats), lam, st,
                                 diag, ptr<int>(h, L.gcnt));
    int rc = fetch_windows(h, p, L, lam, nev);
    if (rc) return rc;
    if (early_t) {
        rc = start_bt2_factors(h, p, L, h->merges_started);
        if (rc) return rc;
    }
    const double ctol = (h->debug & SKEW_EVD_DEBUG_INVIT_NOCONV) ? 0.0 : INVIT_CTOL;
    skew::launch_tridiag_eigvecs(alpha, n, nev, lam, ptr<double>(h, L.stats), ptr<double>(h, L.U0),
                                 ptr<double>(h, L.U1), ptr<double>(h, L.U2), ptr<double>(h, L.Lm),
                                 ptr<unsigned char>(h, L.Sw), ptr<double>(h, L.Yiv), ptr<double>(h, L.ivfac), Q,
                                 ldq, ctol, ptr<unsigned>(h, L.ctl) + CTL_ERR, st, diag);
    HCHK(hipGetLastError());
    rc = tridiag_finish(h, p, L, alpha, nev, lam, Q, ldq, diag);
    if (rc) return rc;
    HCHK(kt_end(h, SKEW_EVD_K_TRIDIAG));
    HCHK(ev_record(h, 4));
    return SKEW_EVD_OK;
}

// After the eigenvalues (lam) and the inverse-iteration vectors (Q): the
// Gram-Schmidt windows and pass, then the degenerate clusters (polished here,
// or flagged on the device in the batched form).
int tridiag_finish(skew_evd_handle h, const Plan &p, const Layout &L, const double *alpha, int nev, double *lam,
                   double *Q, int ldq, const double *diag)
{
    hipStream_t st = h->stream;
    const int n = p.n;
    int rc = plan_windows(h, p, nev);
    if (rc) return rc;
    rc = orthogonalize(h, p, L, Q, ldq, n, nev);
    if (rc) return rc;
    if (h->polish_hi > h->polish_lo) {
        // degenerate clusters: one inverse-iteration step with cluster shifts,
        // then Gram-Schmidt again from the first block they touch
        const int lo = h->polish_lo, m = h->polish_hi - lo;
        HCHK(hipMemcpyAsync(ptr<double>(h, L.pshift), h->lam_host + nev + 1 + lo, sizeof(double) * m,
                            hipMemcpyHostToDevice, st));
        skew::launch_tridiag_polish(alpha, n, m, lam + lo, ptr<double>(h, L.pshift), ptr<double>(h, L.stats),
                                    ptr<double>(h, L.U0), ptr<double>(h, L.U1), ptr<double>(h, L.U2),
                                    ptr<double>(h, L.Lm), ptr<unsigned char>(h, L.Sw), ptr<double>(h, L.Yiv),
                                    ptr<double>(h, L.ivfac), Q + (size_t)lo * ldq, ldq, st, diag);
        HCHK(hipGetLastError());
        rc = orthogonalize(h, p, L, Q, ldq, n, nev, (lo / ORTH_NB) * ORTH_NB);
        if (rc) return rc;
        // the host image of the shifts must outlive the copy
        HCHK(hipStreamSynchronize(st));
    } else if (h->async) {
        skew::launch_degenerate_check(lam, nev, ptr<double>(h, L.stats), DEGEN_TOL, ptr<unsigned>(h, L.ctl) + CTL_FLAGS,
                                      st);
    }
    return SKEW_EVD_OK;
}

// T factors of the stage-2 groups (they depend on the bulge chase only).
template <typename T>
void launch_bt2_factors(skew_evd_handle h, const Plan &p, const Layout &L, hipStream_t st)
{
    const int n = p.n, nev = p.nev, b = p.b;
    if (p.prec && b == 64 && p.nb2 == 64)
        skew::launch_bt2<double>(ptr<double>(h, L.rX), n, n, 2 * nev, b, p.nb2, ptr<double>(h, L.V2),
                                 ptr<double>(h, L.tau2), ptr<double>(h, L.T2), nullptr, ptr<int>(h, L.goff), p.nsig,
                                 p.ngroups, 1, st);
    else
        skew::launch_bt2<T>(ptr<T>(h, L.Z), n, n, 2 * nev, b, p.nb2, ptr<double>(h, L.V2), ptr<double>(h, L.tau2),
                            ptr<T>(h, L.T2), p.prec ? ptr<T>(h, L.V2t) : nullptr, ptr<int>(h, L.goff), p.nsig,
                            p.ngroups, 1, st);
}

// Stage 1 is back-transformed in merged pairs of panels for these widths.
bool merged_bt1(const Plan &p) { return p.b == 64 || p.b == 32; }

// Merged T of each pair of panels (j0, j0 + 1), j0 = P-2, P-4, ...:
// Tm[q] = [[T_j0, -T_j0 G T_j0+1], [0, T_j0+1]], G = V_j0(b:, :)^T V_j0+1,
// with the Gram partials in Gp.
template <typename T>
void launch_bt1_merges(skew_evd_handle h, const Plan &p, const Layout &L, double *Gp, hipStream_t st)
{
    const int n = p.n, b = p.b, P = p.npanels;
    int q = 0;
    for (int j0 = P - 2; j0 >= 0; j0 -= 2, ++q) {
        const int m0 = n - (j0 + 1) * b, m1 = m0 - b;
        const T *V0 = ptr<T>(h, L.Vall) + voff(p, j0);
        const T *V1 = ptr<T>(h, L.Vall) + voff(p, j0 + 1);
        int S = skew::launch_gemm_tn_part<T>(V0 + b, m0, V1, m1, b, b, m1, Gp, st);
        skew::launch_merge_t(ptr<double>(h, L.Tall) + (size_t)j0 * b * b,
                             ptr<double>(h, L.Tall) + (size_t)(j0 + 1) * b * b, Gp, S, b,
                             ptr<double>(h, L.Tm) + (size_t)q * 4 * b * b, st);
    }
}

// Above this order the T factors run on the second stream, beside the
// inverse iteration of the tridiagonal solve (which occupies few CUs).
constexpr int EARLY_TFAC_MIN_N = 4096;

int ensure_aux(skew_evd_handle h)
{
    if (!h->aux) {
        HCHK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
        for (auto &e : h->aux_ev) HCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    return SKEW_EVD_OK;
}

// The merged T of the stage-1 panel pairs on the second stream, once stage 1
// is queued: they depend on stage 1 only and run beside the bulge chase
// (whose workgroups leave CUs free), with their Gram partials in the panel
// path's buffer (free after stage 1).  aux_ev[2] marks them done.
// The caller records aux_ev[3] on the main stream once stage 1 is queued and
// calls this after queueing the chase, so that no work of the main stream is
// submitted behind the merges.
int start_bt1_merges(skew_evd_handle h, const Plan &p, const Layout &L)
{
    HCHK(hipStreamWaitEvent(h->aux, h->aux_ev[3], 0));
    if (p.prec) launch_bt1_merges<float>(h, p, L, ptr<double>(h, L.cqGp), h->aux);
    else launch_bt1_merges<double>(h, p, L, ptr<double>(h, L.cqGp), h->aux);
    HCHK(hipGetLastError());
    HCHK(hipEventRecord(h->aux_ev[2], h->aux));
    return SKEW_EVD_OK;
}

// The T factors of the stage-2 groups on the second stream, once the
// bisection is queued (aux_ev[1] marks them done); merges_started: the
// stage-1 merges were queued there already, else they follow the factors.
int start_bt2_factors(skew_evd_handle h, const Plan &p, const Layout &L, bool merges_started)
{
    int rc = ensure_aux(h);
    if (rc) return rc;
    HCHK(hipEventRecord(h->aux_ev[0], h->stream));
    HCHK(hipStreamWaitEvent(h->aux, h->aux_ev[0], 0));
    if (p.prec) launch_bt2_factors<float>(h, p, L, h->aux);
    else launch_bt2_factors<double>(h, p, L, h->aux);
    HCHK(hipGetLastError());
    HCHK(hipEventRecord(h->aux_ev[1], h->aux));
    if (!merges_started) {
        if (merged_bt1(p)) {
            if (p.prec) launch_bt1_merges<float>(h, p, L, ptr<double>(h, L.cqGp), h->aux);
            else launch_bt1_merges<double>(h, p, L, ptr<double>(h, L.cqGp), h->aux);
            HCHK(hipGetLastError());
        }
        HCHK(hipEventRecord(h->aux_ev[2], h->aux));
    }
    return SKEW_EVD_OK;
}

// early_t: the T factors were started on the second stream after the chase.
template <typename T>
int stage_backtransform(skew_evd_handle h, const Plan &p, const Layout &L, bool early_t)
{
    hipStream_t st = h->stream;
    const int n = p.n, nev = p.nev, b = p.b;
    T *Z = ptr<T>(h, L.Z);
    if (early_t) HCHK(hipStreamWaitEvent(st, h->aux_ev[1], 0));
    // the BT2 timer brackets the application kernel only (D scaling and the
    // T factors of the groups come before it)
    if (p.prec && b == 64 && p.nb2 == 64) {
        // the stage-2 window kernel is FP64-only: apply it to an FP64 copy (in
        // the refinement's X buffer, unused until then) and round once
        double *Zd = ptr<double>(h, L.rX);
        skew::launch_dscale<double>(ptr<double>(h, L.Qd), n, n, nev, Zd, n, st);
        if (!early_t) launch_bt2_factors<T>(h, p, L, st);
        HCHK(kt_begin(h, SKEW_EVD_K_BT2));
        skew::launch_bt2<double>(Zd, n, n, 2 * nev, b, p.nb2, ptr<double>(h, L.V2), ptr<double>(h, L.tau2),
                                 ptr<double>(h, L.T2), nullptr, ptr<int>(h, L.goff), p.nsig, p.ngroups, 2, st);
        HCHK(kt_end(h, SKEW_EVD_K_BT2));
        skew::launch_to_float(Zd, n, (float *)(void *)Z, n, n, 2 * nev, st);
    } else {
        T *V2t = p.prec ? ptr<T>(h, L.V2t) : nullptr;
        skew::launch_dscale<T>(ptr<double>(h, L.Qd), n, n, nev, Z, n, st);
        if (!early_t) launch_bt2_factors<T>(h, p, L, st);
        HCHK(kt_begin(h, SKEW_EVD_K_BT2));
        skew::launch_bt2<T>(Z, n, n, 2 * nev, b, p.nb2, ptr<double>(h, L.V2), ptr<double>(h, L.tau2), ptr<T>(h, L.T2),
                            V2t, ptr<int>(h, L.goff), p.nsig, p.ngroups, 2, st);
        HCHK(kt_end(h, SKEW_EVD_K_BT2));
    }
    HCHK(hipGetLastError());
    HCHK(ev_record(h, 5));
    if (merged_bt1(p)) {
        // consecutive panels merged in pairs: Q_j Q_{j+1} = I - V T V^T with
        // V = [V_j, V_{j+1} shifted by b rows]; pairs end at the last panel
        const int P = p.npanels;
        if (early_t) HCHK(hipStreamWaitEvent(st, h->aux_ev[2], 0));   // merged T factors ready
        else launch_bt1_merges<T>(h, p, L, ptr<double>(h, L.cqGp), st);
        HCHK(kt_begin(h, SKEW_EVD_K_BT1));
        int q = 0;
        for (int j0 = P - 2; j0 >= 0; j0 -= 2, ++q) {
            const int m0 = n - (j0 + 1) * b, m1 = m0 - b;
            const T *V0 = ptr<T>(h, L.Vall) + voff(p, j0);
            const T *V1 = ptr<T>(h, L.Vall) + voff(p, j0 + 1);
            skew::launch_bt1_block<T>(Z, n, (j0 + 1) * b, m0, 2 * nev, V0, b, V1, m1,
                                      ptr<double>(h, L.Tm) + (size_t)q * 4 * b * b, 2 * b, ptr<double>(h, L.Wp),
                                      ptr<T>(h, L.Wt2), st);
            HCHK(hipGetLastError());
        }
        if (P % 2 == 1) {                    // panel 0 alone
            const int m0 = n - b;
            const T *V0 = ptr<T>(h, L.Vall) + voff(p, 0);
            const double *Tf = ptr<double>(h, L.Tall);
            skew::launch_bt1_block<T>(Z, n, b, m0, 2 * nev, V0, b, nullptr, 0, Tf, b, ptr<double>(h, L.Wp),
                                      ptr<T>(h, L.Wt2), st);
            HCHK(hipGetLastError());
        }
        HCHK(kt_end(h, SKEW_EVD_K_BT1));
        HCHK(ev_record(h, 6));
        return SKEW_EVD_OK;
    }
    for (int j = p.npanels - 1; j >= 0; --j) {
        const int r0 = (j + 1) * b, m = n - r0;
        const T *Vd = ptr<T>(h, L.Vall) + voff(p, j);
        const double *Tf = ptr<double>(h, L.Tall) + (size_t)j * b * b;
        HCHK(kt_begin(h, SKEW_EVD_K_BT1));
        int S = skew::launch_gemm_tn_part<T>(Vd, m, Z + r0, n, b, 2 * nev, m, ptr<double>(h, L.Wp), st);
        skew::launch_reduce_left(Tf, ptr<double>(h, L.Wp), S, b, 2 * nev, ptr<double>(h, L.Wt2), st);
        skew::launch_gemm_nn<T>(Vd, m, ptr<double>(h, L.Wt2), 1, m, 2 * nev, b, Z + r0, n, -1.0, 1, st);
        HCHK(kt_end(h, SKEW_EVD_K_BT1));
        HCHK(hipGetLastError());
    }
    HCHK(ev_record(h, 6));
    return SKEW_EVD_OK;
}

int finish_status(skew_evd_handle h, const Layout &L)
{
    unsigned *ctl = ptr<unsigned>(h, L.ctl);
    HCHK(hipMemcpyAsync(h->ctl_host, ctl, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    if (h->ctl_host[CTL_FLAGS] & 1u) return SKEW_EVD_ERR_NONFINITE;
    if (h->ctl_host[CTL_ERR]) {
        const unsigned c = h->ctl_host[CTL_ERR];
        if (c == 8u)
            snprintf(g_errtext, sizeof(g_errtext), "inverse iteration left a vector with residual above %.0e ||T||",
                     INVIT_CTOL);
        else
            snprintf(g_errtext, sizeof(g_errtext), "a device-side wait gave up (code %u)", c);
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

// band widths with a panel kernel instance (band.hip): 8, 16, 32, 64
bool band_supported(int b) { return b == 8 || b == 16 || b == 32 || b == 64; }

int validate_opts(const skew_evd_opts *o)
{
    if (!o) return 0;
    if (o->precision != SKEW_EVD_PREC_FP64 && o->precision != SKEW_EVD_PREC_FP32_REFINE) return 1;
    if (o->tridiag_method != SKEW_EVD_TRIDIAG_BISECT_INVIT) return 1;
    if (o->band != 0 && !band_supported(o->band)) return 1;
    if (o->max_refine_sweeps < 0) return 1;
    if (o->no_fp64_fallback != 0 && o->no_fp64_fallback != 1) return 1;
    if (o->debug & ~(SKEW_EVD_DEBUG_NAN_WS | SKEW_EVD_DEBUG_ZERO_WS | SKEW_EVD_DEBUG_INVIT_NOCONV)) return 1;
    if (o->all_pairs != 0 && o->all_pairs != 1) return 1;
    if (o->panel_method < SKEW_EVD_PANEL_AUTO || o->panel_method > SKEW_EVD_PANEL_HOUSEHOLDER) return 1;
    if (o->reduction != SKEW_EVD_REDUCE_TWO_STAGE && o->reduction != SKEW_EVD_REDUCE_ONE_STAGE &&
        o->reduction != SKEW_EVD_REDUCE_COMPLEX_HERMITIAN)
        return 1;
    // the one-stage routes are FP64 with their own panel width
    if (o->reduction != SKEW_EVD_REDUCE_TWO_STAGE && (o->precision != SKEW_EVD_PREC_FP64 || o->band != 0)) return 1;
    return 0;
}

int solve(skew_evd_handle h, int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr,
          double *Z_im, int ldzi, const skew_evd_opts *opts, skew_evd_info *info);

// Precision form: refine the FP32 pipeline's eigenpairs against the FP64 A.
// Returns OK or WARN_REFINE; results are written to lambda / Z_re / Z_im.
int refine(skew_evd_handle h, const Plan &p, const Layout &L, const double *A, int lda, const skew_evd_opts &o,
           int nev_out, double *lambda, double *Z_re, int ldzr, double *Z_im, int ldzi, int *sweeps_out,
           double *res_out)
{
    hipStream_t st = h->stream;
    const int n = p.n, nev = p.nev;          // the full half: nev = ceil(n/2)
    const int odd = n & 1;
    const int ncx = odd ? 2 * nev - 1 : 2 * nev;
    const int nblk = nev;
    double *X = ptr<double>(h, L.rX), *Xn = ptr<double>(h, L.rXn);
    double *stat = ptr<double>(h, L.rstat);
    skew::launch_build_x<float>(ptr<float>(h, L.Z), n, n, nev, odd, X, st);
    HCHK(hipGetLastError());
    int sweeps = 0;
    double last = 1.0;
    bool converged = false;
    h->refine_passes = 0;
    for (int sw = 0; sw < std::max(1, o.max_refine_sweeps); ++sw) {
        ++h->refine_passes;
        skew::launch_fill32(stat, 0u, 16, st);
        skew::launch_refine_products(A, lda, n, X, ncx, ptr<double>(h, L.rP), ptr<double>(h, L.rS),
                                     ptr<double>(h, L.rG), st);
        skew::launch_refine_eigs(ptr<double>(h, L.rS), ptr<double>(h, L.rG), ncx, nblk, odd, ptr<double>(h, L.rlam),
                                 stat, st);
        HCHK(hipGetLastError());
        double hs[4] = {0, 0, 0, 0};
        HCHK(hipMemcpyAsync(hs, stat, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        const double lmax = hs[2] > 0.0 ? hs[2] : 1.0;
        last = std::max(hs[0], hs[1] / lmax);
        if (last <= o.refine_tol) {
            converged = true;
            break;
        }
        if (o.max_refine_sweeps == 0) break;
        const double omega = 64.0 * 2.220446049250313e-16 * lmax;
        unsigned *nclust = (unsigned *)(stat + 4);
        double *emax = stat + 5;
        skew::launch_refine_update(ptr<double>(h, L.rS), ptr<double>(h, L.rG), n, ncx, nblk, odd,
                                   ptr<double>(h, L.rlam), omega, ptr<float>(h, L.rE), X, Xn, nclust, emax, st);
        HCHK(hipGetLastError());
        double hb[2] = {0.0, 0.0};
        HCHK(hipMemcpyAsync(hb, stat + 4, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        unsigned hc = 0;
        memcpy(&hc, &hb[0], sizeof(unsigned));
        const double ecor = hb[1];
        if (hc) {
            // near-degenerate pairs the FP32 start cannot separate: not refinable
            // here; the outputs get the current iterate X (its eigenvalues are rlam)
            HCHK(hipMemcpyAsync(lambda, ptr<double>(h, L.rlam), sizeof(double) * nev_out, hipMemcpyDeviceToDevice,
                                st));
            skew::launch_split_x(X, n, nev_out, odd, Z_re, ldzr, Z_im, ldzi, st);
            HCHK(hipGetLastError());
            *sweeps_out = sweeps;
            *res_out = last;
            return SKEW_EVD_REFINE_CLUSTER;
        }
        std::swap(X, Xn);
        ++sweeps;
        // a Newton step from an error r whose largest pair correction is e
        // leaves about r * e (r^2 / gap): the quadratic rate holds only for
        // well-separated pairs, so the shortcut takes the correction into account
        if (last * std::max(ecor, last) <= o.refine_tol) {
            converged = true;
            break;
        }
    }
    HCHK(hipMemcpyAsync(lambda, ptr<double>(h, L.rlam), sizeof(double) * nev_out, hipMemcpyDeviceToDevice, st));
    skew::launch_split_x(X, n, nev_out, odd, Z_re, ldzr, Z_im, ldzi, st);
    HCHK(hipGetLastError());
    *sweeps_out = sweeps;
    *res_out = last;
    return converged ? SKEW_EVD_OK : SKEW_EVD_WARN_REFINE;
}

int solve(skew_evd_handle h, int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr,
          double *Z_im, int ldzi, const skew_evd_opts *opts, skew_evd_info *info)
{
    skew_evd_opts o;
    skew_evd_default_opts(&o);
    if (opts) o = *opts;
    const int prec = o.precision;
    const int nev_out = nev;
    // the refinement works on the whole invariant half: the precision form
    // always computes ceil(n/2) pairs and returns the first nev
    if (prec) nev = (n + 1) / 2;
    Plan p = make_plan(n, nev, o.band, prec, o.panel_method, o.reduction == SKEW_EVD_REDUCE_ONE_STAGE,
                       o.reduction == SKEW_EVD_REDUCE_COMPLEX_HERMITIAN);
    Layout L = plan_layout(p);
    int rc = ensure_ws(h, L.total, o.workspace_limit);
    if (rc) return rc;
    hipStream_t st = h->stream;
    h->debug = (unsigned)o.debug;
    kt_reset(h, o.profile != 0, o.profile == 2 ? SKEW_EVD_K_BT2 : -1);
    bool rec[NSTAGE_EV] = {};
    // work left on the second stream by an earlier call that returned early
    if (h->aux) {
        HCHK(hipStreamWaitEvent(st, h->aux_ev[1], 0));
        HCHK(hipStreamWaitEvent(st, h->aux_ev[2], 0));
    }
    h->merges_started = false;
    // test hooks: every workspace byte NaN (0xff) or zero before the solve
    if (o.debug & SKEW_EVD_DEBUG_NAN_WS) skew::launch_fill32(h->ws, 0xffffffffu, h->ws_bytes / 4, st);
    else if (o.debug & SKEW_EVD_DEBUG_ZERO_WS) skew::launch_fill32(h->ws, 0u, h->ws_bytes / 4, st);
    skew::launch_fill32(ptr<unsigned>(h, L.ctl), 0u, 64, st);
    HCHK(ev_record(h, 0));
    rec[0] = true;
    if (p.herm) {
        rc = stage_herm(h, p, L, A, lda);
    } else if (p.onestage) {
        rc = stage_onestage(h, p, L, A, lda);
    } else {
        rc = prec ? stage_band<float>(h, p, L, A, lda, 1) : stage_band<double>(h, p, L, A, lda, 1);
        if (rc) return rc;
        const bool early_m = n >= EARLY_TFAC_MIN_N && p.ngroups > 0 && merged_bt1(p);
        if (early_m) {
            rc = ensure_aux(h);
            if (rc) return rc;
            HCHK(hipEventRecord(h->aux_ev[3], st));   // stage 1 queued
        }
        rc = stage_chase(h, p, L);
        if (rc) return rc;
        if (early_m) {
            rc = start_bt1_merges(h, p, L);
            if (rc) return rc;
            h->merges_started = true;
        }
    }
    if (rc) return rc;
    rec[1] = rec[2] = rec[3] = true;
    const bool early_t = n >= EARLY_TFAC_MIN_N && p.ngroups > 0;
    rc = stage_tridiag(h, p, L, ptr<double>(h, L.alpha), nev, ptr<double>(h, L.lam), ptr<double>(h, L.Qd), n,
                       early_t, p.herm ? ptr<double>(h, L.dgl) : nullptr);
    if (rc) return rc;
    rec[4] = true;
    if (p.herm) rc = stage_bt_herm(h, p, L);
    else if (p.onestage) rc = stage_bt_onestage(h, p, L);
    else rc = prec ? stage_backtransform<float>(h, p, L, early_t) : stage_backtransform<double>(h, p, L, early_t);
    if (rc) return rc;
    rec[5] = rec[6] = true;
    int rsweeps = 0, refine_rc = SKEW_EVD_OK;
    double rres = 0.0;
    if (prec) {
        HCHK(kt_begin(h, SKEW_EVD_K_REFINE));
        refine_rc = refine(h, p, L, A, lda, o, nev_out, lambda, Z_re, ldzr, Z_im, ldzi, &rsweeps, &rres);
        if ((refine_rc == SKEW_EVD_REFINE_CLUSTER || refine_rc == SKEW_EVD_WARN_REFINE) && !o.no_fp64_fallback) {
            // clusters closer than the FP32 pipeline resolves, or no convergence
            // within max_refine_sweeps: fall back to the FP64 form
            skew_evd_opts o64 = o;
            o64.precision = SKEW_EVD_PREC_FP64;
            int rc64 = solve(h, n, A, lda, nev_out, lambda, Z_re, ldzr, Z_im, ldzi, &o64, info);
            if (info) info->refine_sweeps = -1;   // marks the fallback
            return rc64;
        }
        if (refine_rc == SKEW_EVD_REFINE_CLUSTER) refine_rc = SKEW_EVD_WARN_REFINE;
        if (refine_rc != SKEW_EVD_OK && refine_rc != SKEW_EVD_WARN_REFINE) return refine_rc;
        HCHK(kt_end(h, SKEW_EVD_K_REFINE));
    }
    HCHK(ev_record(h, 7));
    rec[7] = true;
    if (!prec) {
        HCHK(hipMemcpyAsync(lambda, ptr<double>(h, L.lam), sizeof(double) * nev, hipMemcpyDeviceToDevice, st));
        const double *Z = ptr<double>(h, L.Z);
        HCHK(hipMemcpy2DAsync(Z_re, sizeof(double) * ldzr, Z, sizeof(double) * n, sizeof(double) * n, nev,
                              hipMemcpyDeviceToDevice, st));
        HCHK(hipMemcpy2DAsync(Z_im, sizeof(double) * ldzi, Z + (size_t)nev * n, sizeof(double) * n,
                              sizeof(double) * n, nev, hipMemcpyDeviceToDevice, st));
    }
    HCHK(ev_record(h, 8));
    rec[8] = true;
    rc = finish_status(h, L);
    if (rc == SKEW_EVD_OK) rc = refine_rc;
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
        info->refine_sweeps = rsweeps;
        info->refine_residual = rres;
        if (prec) {
            // refinement: products (ncx^2 n * 2 + two lower halves) per sweep plus X E
            // per product pass: P = A X (2 n^2 ncx) and the lower halves of X^T P
            // and X^T X (2 ncx^2 n); per update: X E (2 n ncx^2)
            const double nd = n, nc = (n & 1) ? 2.0 * nev - 1.0 : 2.0 * nev;
            info->kern[SKEW_EVD_K_REFINE].flops =
                h->refine_passes * (2.0 * nd * nd * nc + 2.0 * nc * nc * nd) + rsweeps * 2.0 * nd * nc * nc;
        }
        kt_counts(p, info);
        kt_collect(h, info);
    }
    kt_reset(h, false);
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
    opts->max_refine_sweeps = 3;
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
    if (h->ws2) (void)hipFree(h->ws2);
    for (int i = 0; i < NSTAGE_EV; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    if (h->lam_host) (void)hipHostFree(h->lam_host);
    if (h->win_ev) (void)hipEventDestroy(h->win_ev);
    for (auto e : h->kev) (void)hipEventDestroy(e);
    if (h->aux) {
        (void)hipStreamSynchronize(h->aux);
        (void)hipStreamDestroy(h->aux);
    }
    for (auto e : h->aux_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto s2 : h->sub_streams) {
        (void)hipStreamSynchronize(s2);
        (void)hipStreamDestroy(s2);
    }
    for (auto e : h->bev) (void)hipEventDestroy(e);
    if (h->bev0) (void)hipEventDestroy(h->bev0);
    if (h->bhost) (void)hipHostFree(h->bhost);
    if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
    if (h->bstream) {
        (void)hipStreamSynchronize(h->bstream);
        (void)hipStreamDestroy(h->bstream);
    }
    for (auto e : h->bgev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return SKEW_EVD_OK;
}

// ---------------------------------------------------------------------------
// Band-width autotuner.  The band width b (also the panel width of the
// full-to-band stage) trades the MFMA efficiency of the rank-2b updates, which
// grows with b, against the bulge chase and the stage-2 back-transformation,
// whose work grows with b (about 6 n^2 b and 2 n^3 flops in b-long reflector
// groups).  Orders are grouped in classes of TUNE_CLASS; for a class the tuner
// solves a synthetic skew matrix of the class's largest order once per
// candidate band (one warm-up and TUNE_REPS timed calls, wall clock, since
// small solves are bound by their host synchronisations as much as by the
// device) and keeps the fastest.  Results are cached in the handle.
namespace {
constexpr int TUNE_CLASS = 128;
constexpr int TUNE_REPS = 3;
const int TUNE_CAND[] = {16, 32, 64};

int tune_class(int n) { return (n + TUNE_CLASS - 1) / TUNE_CLASS; }

// Synthetic tuning input A = (B - B^T)/2, B with independent entries uniform
// in [-1, 1) from splitmix64 (Steele, Lea and Flood, OOPSLA 2014).
void tune_matrix(int n, std::vector<double> &A)
{
    A.assign((size_t)n * n, 0.0);
    unsigned long long x = 0x5eed5eedULL + (unsigned long long)n;
    auto next = [&]() {
        unsigned long long z = (x += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) {
            const double v = 0.5 * (next() - next());
            A[i + (size_t)j * n] = v;
            A[j + (size_t)i * n] = -v;
        }
}

int tune_band(skew_evd_handle h, int n, int precision, size_t wslimit, int *band, double *ms, int *panel = nullptr)
{
    const int key = precision * 65536 + tune_class(n);
    auto it = h->tune.find(key);
    if (it != h->tune.end()) {
        *band = it->second.band;
        if (panel) *panel = it->second.panel;
        if (ms) *ms = it->second.ms;
        return SKEW_EVD_OK;
    }
    const int nr = tune_class(n) * TUNE_CLASS;
    const int nev = (nr + 1) / 2;
    std::vector<double> hA;
    tune_matrix(nr, hA);
    double *dA = nullptr, *dl = nullptr, *dzr = nullptr, *dzi = nullptr;
    const size_t zb = sizeof(double) * (size_t)nr * nev;
    if (hipMalloc(&dA, sizeof(double) * (size_t)nr * nr) != hipSuccess || hipMalloc(&dl, sizeof(double) * nev) != hipSuccess ||
        hipMalloc(&dzr, zb) != hipSuccess || hipMalloc(&dzi, zb) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(dA);
        (void)hipFree(dl);
        (void)hipFree(dzr);
        (void)hipFree(dzi);
        return SKEW_EVD_ERR_NOMEM;
    }
    int rc = SKEW_EVD_OK;
    hipError_t e = hipMemcpyAsync(dA, hA.data(), sizeof(double) * hA.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        set_hip_error(e, "autotune input copy");
        rc = SKEW_EVD_ERR_HIP;
    }
    int best_b = 0, best_p = SKEW_EVD_PANEL_CHOLQR, last_err = SKEW_EVD_OK;
    double best_ms = 0.0;
    const int ncand = (int)(sizeof(TUNE_CAND) / sizeof(int));
    for (int c = 0; rc == SKEW_EVD_OK && c < 2 * ncand; ++c) {
        const int b = TUNE_CAND[c % ncand];
        const int pm = c < ncand ? SKEW_EVD_PANEL_CHOLQR : SKEW_EVD_PANEL_HOUSEHOLDER;
        if (b > nr - 2) continue;
        skew_evd_opts o;
        skew_evd_default_opts(&o);
        o.precision = precision;
        o.band = b;
        o.panel_method = pm;
        o.workspace_limit = wslimit;
        double tmin = 0.0;
        int crc = SKEW_EVD_OK;
        for (int r = 0; r <= TUNE_REPS && (crc == SKEW_EVD_OK || crc == SKEW_EVD_WARN_REFINE); ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            crc = solve(h, nr, dA, nr, nev, dl, dzr, nr, dzi, nr, &o, nullptr);
            const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (r == 1 || (r > 1 && t < tmin)) tmin = t;
        }
        if (crc != SKEW_EVD_OK && crc != SKEW_EVD_WARN_REFINE) {
            last_err = crc;
            if (crc == SKEW_EVD_ERR_HIP) rc = crc;   // the device is in error: stop
            continue;
        }
        if (best_b == 0 || tmin < best_ms) {
            best_b = b;
            best_p = pm;
            best_ms = tmin;
        }
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(dA);
    (void)hipFree(dl);
    (void)hipFree(dzr);
    (void)hipFree(dzi);
    if (rc) return rc;
    if (best_b == 0) return last_err ? last_err : SKEW_EVD_ERR_NOCONV;
    h->tune[key] = {best_b, best_p, best_ms};
    *band = best_b;
    if (panel) *panel = best_p;
    if (ms) *ms = best_ms;
    return SKEW_EVD_OK;
}
}  // namespace

int skew_evd_autotune(skew_evd_handle h, int n, int precision, int *band, double *ms)
{
    if (!h) return -1;
    if (n < 1 || n > SKEW_EVD_TUNE_NMAX) return -2;
    if (precision != SKEW_EVD_PREC_FP64 && precision != SKEW_EVD_PREC_FP32_REFINE) return -3;
    if (!band) return -4;
    return tune_band(h, n, precision, 0, band, ms);
}

int skew_evd_ex(skew_evd_handle h, int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr,
                double *Z_im, int ldzi, const skew_evd_opts *opts, skew_evd_info *info)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    const bool all = opts && opts->all_pairs == 1;
    if (all ? nev != n : (nev < 0 || nev > (n + 1) / 2)) return -5;
    if (nev > 0 && !lambda) return -6;
    if (nev > 0 && !Z_re) return -7;
    if (ldzr < std::max(1, n)) return -8;
    if (nev > 0 && !Z_im) return -9;
    if (ldzi < std::max(1, n)) return -10;
    if (validate_opts(opts)) return -11;
    if (info) memset(info, 0, sizeof(*info));
    if (n == 0 || nev == 0) return SKEW_EVD_OK;
    skew_evd_opts tuned;
    if (opts && opts->autotune && opts->band == 0 && n <= SKEW_EVD_TUNE_NMAX) {
        int b = 0, pm = SKEW_EVD_PANEL_AUTO;
        int rc = tune_band(h, n, opts->precision, opts->workspace_limit, &b, nullptr, &pm);
        if (rc) return rc;
        tuned = *opts;
        tuned.band = b;
        if (tuned.panel_method == SKEW_EVD_PANEL_AUTO) tuned.panel_method = pm;
        opts = &tuned;
    }
    if (all) {
        // the non-negative half into the last ceil(n/2) columns, then the
        // conjugates of its positive values into the first n - ceil(n/2)
        const int half = (n + 1) / 2, off = n - half;
        int rc = solve(h, n, A, lda, half, lambda + off, Z_re + (size_t)off * ldzr, ldzr, Z_im + (size_t)off * ldzi,
                       ldzi, opts, info);
        if (rc != SKEW_EVD_OK && rc != SKEW_EVD_WARN_REFINE) return rc;
        skew::launch_mirror(Z_re, ldzr, Z_im, ldzi, lambda, n, off, h->stream);
        HCHK(hipGetLastError());
        HCHK(hipStreamSynchronize(h->stream));
        return rc;
    }
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

namespace {

// ---------------------------------------------------------------------------
// Batched form.  Problems up to BATCH_NMAX are solved together, each in its
// own slice of one batch workspace held by the handle:
//   A. on BATCH_STREAMS sub-streams (problems dealt largest first to the
//      least-loaded stream, work ~ n^3): ingest, full-to-band reduction and
//      the chase's preparation;
//   B. one bulge-chase launch for every band: the problems are dealt to up to
//      CHASE_LANES lanes (largest first to the lane with the fewest sweeps)
//      and chased side by side;
//   C. on the sub-streams again: tridiagonal solve, D and both
//      back-transformations, copy-out, and the problem's two status words
//      into a device array.
// No step waits on the host; one synchronisation ends the call.  The orders
// above BATCH_NMAX (whose Gram-Schmidt windows need their eigenvalues on the
// host), and the problems whose spectrum holds a degenerate cluster (their
// eigenvectors need the polishing step, planned on the host), are solved one
// by one afterwards.
constexpr int BATCH_NMAX = 4096;
constexpr int BATCH_STREAMS = 16;
constexpr int CHASE_LANES = 64;

struct BatchItem {
    int idx;
    Plan p;
    Layout L;
    size_t off;
};

// a view of the batch workspace slice of one problem, on a sub-stream
skew_evd_handle_s *make_view(skew_evd_handle h, const BatchItem &it, hipStream_t st)
{
    skew_evd_handle_s *v = new skew_evd_handle_s();
    v->stream = st;
    v->device = h->device;
    v->ws = h->ws + it.off;
    v->ws_bytes = it.L.total;
    v->async = true;
    return v;
}

int batch_part_a(skew_evd_handle v, const BatchItem &it, const double *A, int lda)
{
    skew::launch_fill32(ptr<unsigned>(v, it.L.ctl), 0u, 64, v->stream);
    int rc = stage_band<double>(v, it.p, it.L, A, lda, 1);
    if (rc) return rc;
    chase_prepare(v, it.p, it.L);
    HCHK(hipGetLastError());
    return SKEW_EVD_OK;
}

int batch_part_c(skew_evd_handle v, const BatchItem &it, double *lambda, double *Z_re, double *Z_im,
                 unsigned *stat)
{
    const Plan &p = it.p;
    const Layout &L = it.L;
    const int n = p.n, nev = p.nev;
    hipStream_t st = v->stream;
    // alpha, the eigenvalues and the inverse-iteration vectors come from the
    // batched tridiagonal launches (tri_prob)
    int rc = tridiag_finish(v, p, L, ptr<double>(v, L.alpha), nev, ptr<double>(v, L.lam), ptr<double>(v, L.Qd), n,
                            nullptr);
    if (rc) return rc;
    rc = stage_backtransform<double>(v, p, L, false);
    if (rc) return rc;
    HCHK(hipMemcpyAsync(lambda, ptr<double>(v, L.lam), sizeof(double) * nev, hipMemcpyDeviceToDevice, st));
    const double *Z = ptr<double>(v, L.Z);
    HCHK(hipMemcpyAsync(Z_re, Z, sizeof(double) * n * nev, hipMemcpyDeviceToDevice, st));
    HCHK(hipMemcpyAsync(Z_im, Z + (size_t)nev * n, sizeof(double) * n * nev, hipMemcpyDeviceToDevice, st));
    HCHK(hipMemcpyAsync(stat, ptr<unsigned>(v, L.ctl), sizeof(unsigned) * 2, hipMemcpyDeviceToDevice, st));
    return SKEW_EVD_OK;
}

// The problem's entry of the batched tridiagonal launches (its workspace
// slice starts at w).
skew::TriProb tri_prob(char *w, const BatchItem &it)
{
    const Plan &p = it.p;
    const Layout &L = it.L;
    skew::TriProb t{};
    t.ab = (const double *)(w + L.ab);
    t.alpha = (double *)(w + L.alpha);
    t.a2 = (double *)(w + L.a2);
    t.stats = (double *)(w + L.stats);
    t.w = (double *)(w + L.lam);
    t.U0 = (double *)(w + L.U0);
    t.U1 = (double *)(w + L.U1);
    t.U2 = (double *)(w + L.U2);
    t.Lm = (double *)(w + L.Lm);
    t.Y = (double *)(w + L.Yiv);
    t.fac = (double *)(w + L.ivfac);
    t.Q = (double *)(w + L.Qd);
    t.Sw = (unsigned char *)(w + L.Sw);
    t.err = (unsigned *)(w + L.ctl) + CTL_ERR;
    t.gcnt = (int *)(w + L.gcnt);
    t.diag = nullptr;
    t.shifts = nullptr;
    t.ctol = INVIT_CTOL;
    t.ldab = 2 * p.b + 1;
    t.n = p.n;
    t.first = p.n / 2;
    t.nev = p.nev;
    t.ldq = p.n;
    t.iters = 2;
    return t;
}

int ensure_streams(skew_evd_handle h, int S)
{
    while ((int)h->sub_streams.size() < S) {
        hipStream_t s2;
        HCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        h->sub_streams.push_back(s2);
        hipEvent_t e;
        HCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->bev.push_back(e);
    }
    if (!h->bev0) HCHK(hipEventCreateWithFlags(&h->bev0, hipEventDisableTiming));
    if (!h->bstream) HCHK(hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking));
    for (auto &e : h->bgev)
        if (!e) HCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return SKEW_EVD_OK;
}

// the sub-streams 0..S-1 wait for the work queued on ms
int fork_streams(skew_evd_handle h, hipStream_t ms, int S)
{
    HCHK(hipEventRecord(h->bev0, ms));
    for (int k = 0; k < S; ++k) HCHK(hipStreamWaitEvent(h->sub_streams[k], h->bev0, 0));
    return SKEW_EVD_OK;
}

// ms waits for the work queued on the sub-streams 0..S-1
int join_streams(skew_evd_handle h, hipStream_t ms, int S)
{
    for (int k = 0; k < S; ++k) {
        HCHK(hipEventRecord(h->bev[k], h->sub_streams[k]));
        HCHK(hipStreamWaitEvent(ms, h->bev[k], 0));
    }
    return SKEW_EVD_OK;
}

// Problems whose spectrum holds a degenerate cluster (flagged on the device)
// are appended to `again`, to be solved on their own.
int batched_together(skew_evd_handle h, const std::vector<int> &ids, const int *n, const double *const *A,
                     const int *lda, const int *nev, double *const *lambda, double *const *Z_re,
                     double *const *Z_im, const std::vector<skew_evd_opts> &popt, size_t wslimit, int *status,
                     std::vector<int> &again)
{
    const int cnt = (int)ids.size();
    if (cnt == 0) return SKEW_EVD_OK;
    std::vector<BatchItem> it(cnt);
    size_t off = 0;
    for (int k = 0; k < cnt; ++k) {
        const int i = ids[k];
        it[k].idx = i;
        it[k].p = make_plan(n[i], nev[i], popt[i].band, 0, popt[i].panel_method);
        it[k].L = plan_layout(it[k].p);
        it[k].off = off;
        off += it[k].L.total;
    }
    const int M = std::min(cnt, CHASE_LANES);
    const size_t probs_off = off;
    off += al(sizeof(skew::ChaseProb) * cnt);
    const size_t tri_off = off;
    off += al(sizeof(skew::TriProb) * cnt);
    const size_t lanes_off = off;
    off += al(sizeof(int) * (M + 1 + 2 * cnt));
    const size_t pre_off = off;
    off += al(sizeof(int) * 3 * (cnt + 1));
    const size_t stat_off = off;
    off += al(sizeof(unsigned) * (2 * cnt + 2));
    int rc = ensure_ws(h, off, wslimit);
    if (rc) return rc;
    const int S = std::min(cnt, BATCH_STREAMS);
    rc = ensure_streams(h, S);
    if (rc) return rc;
    // streams (LPT on n^3) and chase lanes (LPT on sweeps)
    std::vector<int> order(cnt);
    for (int k = 0; k < cnt; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return it[a].p.n > it[b].p.n; });
    std::vector<std::vector<int>> part(S), lane(M);
    std::vector<double> load(S, 0.0);
    std::vector<long> lload(M, 0);
    for (int k : order) {
        const int s2 = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        part[s2].push_back(k);
        const double nn = it[k].p.n;
        load[s2] += nn * nn * nn + 1e6;
        const int l = (int)(std::min_element(lload.begin(), lload.end()) - lload.begin());
        lane[l].push_back(k);
        lload[l] += std::max(it[k].p.n - 2, 0);
    }
    // host images of the chase and tridiagonal descriptors, then one copy
    // each to the device
    const size_t hbytes = sizeof(skew::ChaseProb) * cnt + sizeof(skew::TriProb) * cnt +
                          sizeof(int) * (M + 1 + 2 * cnt) + sizeof(int) * 3 * (cnt + 1) +
                          sizeof(unsigned) * (2 * cnt + 2);
    if (hbytes > h->bhost_cap) {
        if (h->bhost) {
            // a replay of the previous batch may still read the old images
            HCHK(hipStreamSynchronize(h->bstream));
            HCHK(hipHostFree(h->bhost));
        }
        h->bhost = nullptr;
        h->bhost_cap = 0;
        HCHK(hipHostMalloc((void **)&h->bhost, hbytes, hipHostMallocDefault));
        h->bhost_cap = hbytes;
        ++h->bhost_gen;
    }
    skew::ChaseProb *hp = (skew::ChaseProb *)h->bhost;
    skew::TriProb *ht = (skew::TriProb *)(hp + cnt);
    int *hl = (int *)(ht + cnt);
    int *hpre = hl + M + 1 + 2 * cnt;
    unsigned *hs = (unsigned *)(hpre + 3 * (cnt + 1));
    int maxlen = 0, nitem = 0;
    for (int l = 0; l < M; ++l) {
        hl[l] = nitem;
        int pos = 0;
        for (int k : lane[l]) {
            hl[M + 1 + 2 * nitem] = k;
            hl[M + 1 + 2 * nitem + 1] = pos;
            ++nitem;
            pos += std::max(it[k].p.n - 2, 0);
        }
        maxlen = std::max(maxlen, pos);
    }
    hl[M] = nitem;
    for (int k = 0; k < cnt; ++k) {
        const Plan &p = it[k].p;
        const Layout &L = it[k].L;
        char *w = h->ws + it[k].off;
        unsigned *ctl = (unsigned *)(w + L.ctl);
        hp[k] = skew::ChaseProb{(double *)(w + L.ab), (double *)(w + L.V2), (double *)(w + L.tau2),
                                (const int *)(w + L.goff), ctl + CTL_PROGRESS, ctl + CTL_ERR, 2 * p.b + 1, p.n,
                                p.b, p.nb2};
        ht[k] = tri_prob(w, it[k]);
    }
    // workgroups per problem of the batched bisection, inverse iteration and
    // transposition: prefix tables
    int tot[3] = {0, 0, 0};
    for (int t = 0; t < 3; ++t) {
        int *pt = hpre + t * (cnt + 1);
        pt[0] = 0;
        for (int k = 0; k < cnt; ++k) {
            const int nn = it[k].p.n, ne = it[k].p.nev;
            const int gk = (t == 0) ? skew::tri_bisect_groups(ne)
                                    : ((t == 1) ? skew::tri_invit_groups(ne) : skew::tri_transpose_groups(nn, ne));
            pt[k + 1] = pt[k] + gk;
        }
        tot[t] = pt[cnt];
    }
    skew::ChaseProb *dprobs = (skew::ChaseProb *)(h->ws + probs_off);
    skew::TriProb *dtri = (skew::TriProb *)(h->ws + tri_off);
    int *dlanes = (int *)(h->ws + lanes_off);
    int *dpre = (int *)(h->ws + pre_off);
    unsigned *dstat = (unsigned *)(h->ws + stat_off);
    // The launch sequence depends on nothing but this key.  Its first call
    // captures the sequence as a HIP graph (on bstream, which can be
    // captured whatever h->stream is); later calls with the same key replay
    // the graph, which spares the host the enqueueing of every launch.
    std::vector<uintptr_t> key = {(uintptr_t)h->ws,   (uintptr_t)h->ws_gen, (uintptr_t)h->bhost,
                                  (uintptr_t)h->bhost_gen, (uintptr_t)cnt, (uintptr_t)S,
                                  (uintptr_t)M,       (uintptr_t)maxlen};
    for (int k = 0; k < cnt; ++k) {
        const int i = it[k].idx;
        const Plan &p = it[k].p;
        for (uintptr_t x : {(uintptr_t)p.n, (uintptr_t)p.nev, (uintptr_t)p.b, (uintptr_t)p.hh_panels,
                            (uintptr_t)A[i], (uintptr_t)lda[i], (uintptr_t)lambda[i], (uintptr_t)Z_re[i],
                            (uintptr_t)Z_im[i], (uintptr_t)it[k].off})
            key.push_back(x);
    }
    const hipStream_t ms = h->bstream;
    if (!(h->bgraph && key == h->bkey)) {
        if (h->bgraph) {
            HCHK(hipStreamSynchronize(ms));
            HCHK(hipGraphExecDestroy(h->bgraph));
            h->bgraph = nullptr;
            h->bkey.clear();
        }
        std::vector<skew_evd_handle_s *> views(cnt);
        for (int s2 = 0; s2 < S; ++s2)
            for (int k : part[s2]) views[k] = make_view(h, it[k], h->sub_streams[s2]);
        // One host thread enqueues everything, taking the streams in turn
        // (problem r of every stream, then problem r + 1, ...).  (With one
        // enqueueing thread per stream, the launches of several threads met
        // inside the runtime, and a profiler's interception of them crashed.)
        std::vector<int> src(S, SKEW_EVD_OK);
        size_t rounds = 0;
        for (int s2 = 0; s2 < S; ++s2) rounds = std::max(rounds, part[s2].size());
        auto run_parts = [&](bool first) {
            for (size_t r = 0; r < rounds; ++r)
                for (int s2 = 0; s2 < S; ++s2) {
                    if (r >= part[s2].size() || src[s2]) continue;
                    const int k = part[s2][r], i = it[k].idx;
                    src[s2] = first ? batch_part_a(views[k], it[k], A[i], lda[i])
                                    : batch_part_c(views[k], it[k], lambda[i], Z_re[i], Z_im[i], dstat + 2 * k);
                }
        };
        auto enqueue = [&]() -> int {
            HCHK(hipMemcpyAsync(dprobs, hp, sizeof(skew::ChaseProb) * cnt, hipMemcpyHostToDevice, ms));
            HCHK(hipMemcpyAsync(dtri, ht, sizeof(skew::TriProb) * cnt, hipMemcpyHostToDevice, ms));
            HCHK(hipMemcpyAsync(dlanes, hl, sizeof(int) * (M + 1 + 2 * cnt), hipMemcpyHostToDevice, ms));
            HCHK(hipMemcpyAsync(dpre, hpre, sizeof(int) * 3 * (cnt + 1), hipMemcpyHostToDevice, ms));
            skew::launch_fill32(dstat, 0u, 2 * (size_t)cnt + 2, ms);
            int r2 = fork_streams(h, ms, S);
            if (r2) return r2;
            run_parts(true);
            r2 = join_streams(h, ms, S);
            for (int s2 = 0; s2 < S && !r2; ++s2) r2 = src[s2];
            if (r2) return r2;
            const int G = std::max(1, std::min(skew::chase_max_workgroups(), 8 * M));
            HCHK(skew::launch_chase_batched(dprobs, dlanes, M, maxlen, G, dstat + 2 * cnt, ms));
            skew::launch_tridiag_batched(dtri, dpre, cnt, tot, ms);
            HCHK(hipGetLastError());
            r2 = fork_streams(h, ms, S);
            if (r2) return r2;
            run_parts(false);
            r2 = join_streams(h, ms, S);
            for (int s2 = 0; s2 < S && !r2; ++s2) r2 = src[s2];
            return r2;
        };
        HCHK(hipStreamBeginCapture(ms, hipStreamCaptureModeRelaxed));
        rc = enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ms, &g);
        for (auto v : views) delete v;
        if (!rc && ec != hipSuccess) {
            snprintf(g_errtext, sizeof(g_errtext), "capture of the batch: %s", hipGetErrorString(ec));
            rc = SKEW_EVD_ERR_HIP;
        }
        if (!rc) {
            const hipError_t ei = hipGraphInstantiate(&h->bgraph, g, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                snprintf(g_errtext, sizeof(g_errtext), "instantiation of the batch graph: %s",
                         hipGetErrorString(ei));
                h->bgraph = nullptr;
                rc = SKEW_EVD_ERR_HIP;
            }
        }
        if (g) (void)hipGraphDestroy(g);
        if (rc) {
            (void)hipGetLastError();
            return rc;
        }
        h->bkey = key;
    }
    // ordered after the work already on h->stream, and h->stream after it
    HCHK(hipEventRecord(h->bgev[0], h->stream));
    HCHK(hipStreamWaitEvent(ms, h->bgev[0], 0));
    HCHK(hipGraphLaunch(h->bgraph, ms));
    HCHK(hipEventRecord(h->bgev[1], ms));
    HCHK(hipStreamWaitEvent(h->stream, h->bgev[1], 0));
    HCHK(hipMemcpyAsync(hs, dstat, sizeof(unsigned) * 2 * cnt, hipMemcpyDeviceToHost, h->stream));
    HCHK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < cnt; ++k) {
        const int i = it[k].idx;
        if (hs[2 * k] & 1u) status[i] = SKEW_EVD_ERR_NONFINITE;
        else if (hs[2 * k + 1]) status[i] = SKEW_EVD_ERR_NOCONV;
        else status[i] = SKEW_EVD_OK;
        if (status[i] == SKEW_EVD_OK && (hs[2 * k] & 2u)) again.push_back(i);
    }
    return SKEW_EVD_OK;
}

}  // namespace

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
    // the precision form and the one-stage route are not available in the
    // batched form (see the header)
    if (opts && (opts->precision != SKEW_EVD_PREC_FP64 || opts->reduction != SKEW_EVD_REDUCE_TWO_STAGE)) return -10;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0) return -3;
        if (n[i] > 0 && !A[i]) return -4;
        if (lda[i] < std::max(1, n[i])) return -5;
        if (nev[i] < 0 || nev[i] > (n[i] + 1) / 2) return -6;
        if (nev[i] > 0 && !lambda[i]) return -7;
        if (nev[i] > 0 && !Z_re[i]) return -8;
        if (nev[i] > 0 && !Z_im[i]) return -9;
    }
    if (info) memset(info, 0, sizeof(*info));
    if (count == 0) return SKEW_EVD_OK;
    // autotuned band widths: each size class is tuned once on h, before any
    // problem is solved
    std::vector<skew_evd_opts> popt(count);
    for (int i = 0; i < count; ++i) {
        if (opts) popt[i] = *opts;
        else skew_evd_default_opts(&popt[i]);
        if (popt[i].autotune && popt[i].band == 0 && n[i] >= 1 && n[i] <= SKEW_EVD_TUNE_NMAX) {
            int b = 0, pm = SKEW_EVD_PANEL_AUTO;
            int rc = tune_band(h, n[i], popt[i].precision, popt[i].workspace_limit, &b, nullptr, &pm);
            if (rc) {
                // nothing was solved: every problem reports the tuner's status
                for (int k = 0; k < count; ++k) status[k] = rc;
                return rc;
            }
            popt[i].band = b;
            if (popt[i].panel_method == SKEW_EVD_PANEL_AUTO) popt[i].panel_method = pm;
        }
        popt[i].autotune = 0;
    }
    const size_t wslimit = opts ? opts->workspace_limit : 0;
    std::vector<int> together, alone;
    for (int i = 0; i < count; ++i) {
        status[i] = SKEW_EVD_OK;
        if (n[i] == 0 || nev[i] == 0) continue;
        (n[i] <= BATCH_NMAX ? together : alone).push_back(i);
    }
    HCHK(hipEventRecord(h->ev[0], h->stream));
    int rc = batched_together(h, together, n, A, lda, nev, lambda, Z_re, Z_im, popt, wslimit, status, alone);
    if (rc) {
        for (int i : together) status[i] = rc;
        return rc;
    }
    for (int i : alone)
        status[i] = skew_evd_ex(h, n[i], A[i], lda[i], nev[i], lambda[i], Z_re[i], std::max(1, n[i]), Z_im[i],
                                std::max(1, n[i]), &popt[i], nullptr);
    HCHK(hipEventRecord(h->ev[8], h->stream));
    HCHK(hipEventSynchronize(h->ev[8]));
    int first = 0;
    for (int i = 0; i < count; ++i)
        if (status[i] && !first) first = status[i];
    if (info) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[0], h->ev[8]) == hipSuccess) info->ms_total = ms;
        info->workspace_bytes = h->ws_bytes;
        info->band = together.empty() ? 0 : make_plan(n[together[0]], nev[together[0]], popt[together[0]].band, 0).b;
    }
    return first;
}

// ---------------------------------------------------------------------------
// Allocation-free entry point.  Its workspace is the file-scope device array
// `scratch`; each device that runs it holds its own copy from the first call
// until the process ends.  The array's device address on a device is taken
// once, with that device current, through hipGetSymbolAddress and kept per
// device: host code never passes the array's name itself (a host-side stand-in,
// not a device address).  The host-side state of a call (control words and
// eigenvalues read back, the stage drivers' bookkeeping) is also fixed
// storage, one slot per device, so calls on one device must not overlap.
static __device__ __align__(256) char scratch[SKEW_EVD_NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAXDEV = 64;
struct NoallocSlot {
    char *ws = nullptr;                  // device address of `scratch` on this device
    skew_evd_handle_s h;
    unsigned ctl[64];
    double lam[2 * SKEW_EVD_NOALLOC_NMAX + 1];
};
NoallocSlot g_noalloc[NOALLOC_MAXDEV];
}  // namespace

int skew_evd_noalloc(int n, const double *A, int lda, int nev, double *lambda, double *Z_re, int ldzr, double *Z_im,
                     int ldzi, void *hip_stream)
{
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max(1, n)) return -3;
    if (nev < 0 || nev > (n + 1) / 2) return -4;
    if (nev > 0 && !lambda) return -5;
    if (nev > 0 && !Z_re) return -6;
    if (ldzr < std::max(1, n)) return -7;
    if (nev > 0 && !Z_im) return -8;
    if (ldzi < std::max(1, n)) return -9;
    if (n > SKEW_EVD_NOALLOC_NMAX) {
        snprintf(g_errtext, sizeof(g_errtext), "n = %d exceeds the allocation-free limit n <= %d", n,
                 SKEW_EVD_NOALLOC_NMAX);
        return SKEW_EVD_ERR_NOMEM;
    }
    if (n == 0 || nev == 0) return SKEW_EVD_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAXDEV) {
        (void)hipGetLastError();
        snprintf(g_errtext, sizeof(g_errtext), "no usable HIP device");
        return SKEW_EVD_ERR_NODEVICE;
    }
    NoallocSlot &sl = g_noalloc[dev];
    if (!sl.ws) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_hip_error(e, "hipGetSymbolAddress(scratch)");
            return SKEW_EVD_ERR_HIP;
        }
        sl.ws = (char *)p;
        sl.h.device = dev;
        sl.h.noalloc = true;
        sl.h.ctl_host = sl.ctl;
        sl.h.lam_host = sl.lam;
        sl.h.lam_cap = 2 * SKEW_EVD_NOALLOC_NMAX + 1;
    }
    sl.h.ws = sl.ws;
    sl.h.ws_bytes = SKEW_EVD_NOALLOC_BYTES;
    sl.h.stream = (hipStream_t)hip_stream;
    skew_evd_opts o;
    skew_evd_default_opts(&o);
    o.workspace_limit = SKEW_EVD_NOALLOC_BYTES;
    const Plan p = make_plan(n, nev, 0, SKEW_EVD_PREC_FP64);
    if (plan_layout(p).total > SKEW_EVD_NOALLOC_BYTES) {
        snprintf(g_errtext, sizeof(g_errtext), "workspace of n = %d exceeds the allocation-free array", n);
        return SKEW_EVD_ERR_NOMEM;
    }
    return solve(&sl.h, n, A, lda, nev, lambda, Z_re, ldzr, Z_im, ldzi, &o, nullptr);
}

// ---------------------------------------------------------------------------
// The Bethe-Salpeter route (Section 3): M, Cholesky, the skew eigenproblem of
// L^T J L through solve(), and the back-transformation of its vectors.
int skew_evd_bse(skew_evd_handle h, int m, const double *A_re, const double *A_im, int lda, const double *B_re,
                 const double *B_im, int ldb, int nev, double *lambda, double *X_re, double *X_im, int ldx,
                 const skew_evd_opts *opts, skew_evd_info *info)
{
    if (!h) return -1;
    if (m < 0) return -2;
    if (m > 0 && !A_re) return -3;
    if (m > 0 && !A_im) return -4;
    if (lda < std::max(1, m)) return -5;
    if (m > 0 && !B_re) return -6;
    if (m > 0 && !B_im) return -7;
    if (ldb < std::max(1, m)) return -8;
    if (nev < 0 || nev > m) return -9;
    if (nev > 0 && !lambda) return -10;
    if (nev > 0 && !X_re) return -11;
    if (nev > 0 && !X_im) return -12;
    if (ldx < std::max(1, 2 * m)) return -13;
    if (validate_opts(opts) || (opts && opts->all_pairs)) return -14;
    if (info) memset(info, 0, sizeof(*info));
    if (m == 0 || nev == 0) return SKEW_EVD_OK;
    const int n = 2 * m;
    const size_t nblk = (n + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al(bytes);
        return o;
    };
    const size_t oM = take(sizeof(double) * (size_t)n * n), oK = take(sizeof(double) * (size_t)n * n),
                 oR = take(sizeof(double) * nblk * 64 * 64), oZ = take(sizeof(double) * (size_t)n * 2 * nev),
                 oW = take(sizeof(double) * (size_t)tn_parts_max() * 64 * 2 * nev), oF = take(sizeof(unsigned) * 4);
    const size_t limit = opts ? opts->workspace_limit : 0;
    if (limit && off > limit) {
        snprintf(g_errtext, sizeof(g_errtext), "workspace of %zu bytes exceeds the limit of %zu", off, limit);
        return SKEW_EVD_ERR_NOMEM;
    }
    if (off > h->ws2_bytes) {
        HCHK(hipStreamSynchronize(h->stream));
        if (h->ws2) HCHK(hipFree(h->ws2));
        h->ws2 = nullptr;
        h->ws2_bytes = 0;
        if (hipMalloc((void **)&h->ws2, off) != hipSuccess) {
            (void)hipGetLastError();
            h->ws2 = nullptr;
            snprintf(g_errtext, sizeof(g_errtext), "hipMalloc of %zu bytes failed", off);
            return SKEW_EVD_ERR_NOMEM;
        }
        h->ws2_bytes = off;
    }
    hipStream_t st = h->stream;
    double *M = (double *)(h->ws2 + oM), *K = (double *)(h->ws2 + oK), *Rinv = (double *)(h->ws2 + oR),
           *Z = (double *)(h->ws2 + oZ), *Wp = (double *)(h->ws2 + oW);
    unsigned *flags = (unsigned *)(h->ws2 + oF);
    skew::launch_fill32(flags, 0u, 4, st);
    skew::launch_bse_build_m(A_re, A_im, lda, B_re, B_im, ldb, m, M, n, flags, st);
    skew::launch_cholesky(M, n, n, Rinv, flags, st);
    HCHK(hipGetLastError());
    unsigned hf[4] = {0, 0, 0, 0};
    HCHK(hipMemcpyAsync(hf, flags, sizeof(unsigned) * 4, hipMemcpyDeviceToHost, st));
    HCHK(hipStreamSynchronize(st));
    if (hf[0] & 1u) return SKEW_EVD_ERR_NONFINITE;
    if (hf[0] & 4u) return SKEW_EVD_ERR_NOTDEF;
    skew::launch_ltjl(M, n, m, K, n, st);
    HCHK(hipGetLastError());
    int rc = solve(h, n, K, n, nev, lambda, Z, n, Z + (size_t)n * nev, n, opts, info);
    if (rc != SKEW_EVD_OK && rc != SKEW_EVD_WARN_REFINE) return rc;
    skew::launch_trsm_lt(M, n, n, Rinv, Z, n, 2 * nev, Wp, st);
    skew::launch_bse_x(Z, n, m, nev, lambda, X_re, X_im, ldx, st);
    HCHK(hipGetLastError());
    HCHK(hipStreamSynchronize(st));
    return rc;
}

int skew_evd_band_reduce(skew_evd_handle h, int n, const double *A, int lda, int b, double *band, int ldband)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max(1, n)) return -4;
    if (!band_supported(b)) return -5;
    if (n > 0 && !band) return -6;
    if (ldband < b + 1) return -7;
    if (n == 0) return SKEW_EVD_OK;
    Plan p = make_plan(n, 0, b, 0);
    Layout L = plan_layout(p);
    kt_reset(h, false);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    skew::launch_fill32(ptr<unsigned>(h, L.ctl), 0u, 64, h->stream);
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
    if (b != 0 && !band_supported(b)) return -5;
    if (n > 1 && !alpha) return -6;
    if (n <= 1) return SKEW_EVD_OK;
    Plan p = make_plan(n, 0, b, 0);
    Layout L = plan_layout(p);
    kt_reset(h, false);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    skew::launch_fill32(ptr<unsigned>(h, L.ctl), 0u, 64, h->stream);
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
    kt_reset(h, false);
    int rc = ensure_ws(h, L.total, 0);
    if (rc) return rc;
    skew::launch_fill32(ptr<unsigned>(h, L.ctl), 0u, 64, h->stream);
    if (n == 1) {
        skew::launch_fill32(ptr<double>(h, L.alpha), 0u, 2, h->stream);
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
    case SKEW_EVD_ERR_NOTDEF: return "the Bethe-Salpeter matrix is not definite (Cholesky of M failed)";
    default: return status < 0 ? "invalid argument" : "unknown status";
    }
}

int skew_evd_version(void) { return 100; }

}  // extern "C"
