"""Python binding of the skew-symmetric eigensolver library (libskewevd.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI of include/skew_evd.h.  PyTorch supplies device
memory and the current stream.  The library must have been built (see
paper_1912_04062_amd/build.py); importing this module without it raises.
"""
import atexit
import ctypes
import os
import sys
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskewevd.so")

OK = 0
ERR_NONFINITE = 1
ERR_NOCONV = 2
WARN_REFINE = 3
ERR_NOMEM = 4
ERR_HIP = 5
ERR_NODEVICE = 6
ERR_NOTDEF = 7

PREC_FP64 = 0
PREC_FP32_REFINE = 1

DEBUG_NAN_WS = 1
DEBUG_ZERO_WS = 2
DEBUG_INVIT_NOCONV = 4
_PREC = {"fp64": PREC_FP64, "fp32": PREC_FP32_REFINE, "fp32_refine": PREC_FP32_REFINE}
REDUCE_TWO_STAGE = 0
REDUCE_ONE_STAGE = 1
REDUCE_COMPLEX_HERMITIAN = 2
_REDUCE = {"two": REDUCE_TWO_STAGE, "one": REDUCE_ONE_STAGE, "complex": REDUCE_COMPLEX_HERMITIAN}


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("band", ctypes.c_int),
                ("max_refine_sweeps", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("workspace_limit", ctypes.c_size_t), ("profile", ctypes.c_int),
                ("autotune", ctypes.c_int), ("no_fp64_fallback", ctypes.c_int),
                ("debug", ctypes.c_int), ("all_pairs", ctypes.c_int), ("panel_method", ctypes.c_int),
                ("reduction", ctypes.c_int), ("tridiag_method", ctypes.c_int)]


class KStat(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("launches", ctypes.c_int), ("bound", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_stage", ctypes.c_double * 8),
                ("band", ctypes.c_int), ("refine_sweeps", ctypes.c_int),
                ("refine_residual", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t),
                ("kern", KStat * 8)]

    STAGES = ("ingest", "full_to_band", "bulge_chase", "tridiag_solve", "bt2", "bt1",
              "refine", "copy_out")
    KERNELS = ("panel_qr", "skew_symm_w", "skew_syr2k", "bulge_chase", "tridiag", "bt2", "bt1",
               "refine")
    BOUNDS = ("mfma", "hbm", "alu")

    def as_dict(self):
        d = {"ms_total": self.ms_total, "band": self.band, "refine_sweeps": self.refine_sweeps,
             "refine_residual": self.refine_residual, "workspace_bytes": int(self.workspace_bytes)}
        d["ms_stage"] = {k: self.ms_stage[i] for i, k in enumerate(self.STAGES)}
        d["kernels"] = {k: {"ms": self.kern[i].ms, "flops": self.kern[i].flops,
                            "bytes": self.kern[i].bytes, "launches": self.kern[i].launches,
                            "bound": self.BOUNDS[self.kern[i].bound]}
                        for i, k in enumerate(self.KERNELS)}
        return d


class SkewEvdError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: status {status}: {status_string(status)}")


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1912_04062_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.skew_evd_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.skew_evd_default_opts.restype = None
    lib.skew_evd_create.argtypes = [ctypes.POINTER(vp), vp]
    lib.skew_evd_create.restype = ip
    lib.skew_evd_destroy.argtypes = [vp]
    lib.skew_evd_destroy.restype = ip
    lib.skew_evd_ex.argtypes = [vp, ip, vp, ip, ip, vp, vp, ip, vp, ip, ctypes.POINTER(Opts),
                                ctypes.POINTER(Info)]
    lib.skew_evd_ex.restype = ip
    lib.skew_evd.argtypes = [ip, vp, ip, ip, vp, vp, vp]
    lib.skew_evd.restype = ip
    lib.skew_evd_batched.argtypes = [vp, ip, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Opts),
                                     ctypes.POINTER(Info), vp]
    lib.skew_evd_batched.restype = ip
    lib.skew_evd_band_reduce.argtypes = [vp, ip, vp, ip, ip, vp, ip]
    lib.skew_evd_band_reduce.restype = ip
    lib.skew_evd_tridiagonalize.argtypes = [vp, ip, vp, ip, ip, vp]
    lib.skew_evd_tridiagonalize.restype = ip
    lib.skew_evd_tridiag_eig.argtypes = [vp, ip, vp, ip, vp, vp, ip]
    lib.skew_evd_tridiag_eig.restype = ip
    lib.skew_evd_status_string.argtypes = [ip]
    lib.skew_evd_status_string.restype = ctypes.c_char_p
    lib.skew_evd_autotune.argtypes = [vp, ip, ip, ctypes.POINTER(ip), ctypes.POINTER(ctypes.c_double)]
    lib.skew_evd_autotune.restype = ip
    lib.skew_evd_version.argtypes = []
    lib.skew_evd_version.restype = ip
    lib.skew_evd_noalloc.argtypes = [ip, vp, ip, ip, vp, vp, ip, vp, ip, vp]
    lib.skew_evd_noalloc.restype = ip
    lib.skew_evd_bse.argtypes = [vp, ip, vp, vp, ip, vp, vp, ip, ip, vp, vp, vp, ip, ctypes.POINTER(Opts),
                                 ctypes.POINTER(Info)]
    lib.skew_evd_bse.restype = ip
    _lib = lib
    return lib


def lib():
    return _load()


def status_string(status):
    return _load().skew_evd_status_string(int(status)).decode()


def default_opts(precision="fp64", band=0, max_refine_sweeps=None, refine_tol=None,
                 workspace_limit=0, profile=0, autotune=0, no_fp64_fallback=0, debug=0, all_pairs=0,
                 panel_method=0, reduction=0):
    o = Opts()
    _load().skew_evd_default_opts(ctypes.byref(o))
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.band = int(band)
    if max_refine_sweeps is not None:
        o.max_refine_sweeps = int(max_refine_sweeps)
    if refine_tol is not None:
        o.refine_tol = float(refine_tol)
    o.workspace_limit = int(workspace_limit)
    o.profile = int(profile)
    o.autotune = int(autotune)
    o.no_fp64_fallback = int(no_fp64_fallback)
    o.debug = int(debug)
    o.all_pairs = int(all_pairs)
    o.panel_method = int(panel_method)
    o.reduction = _REDUCE[reduction] if isinstance(reduction, str) else int(reduction)
    return o


def colmajor(A):
    """(tensor, ld) whose memory holds A column-major (a copy unless it already does)."""
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    n, m = A.shape
    if A.stride(0) == 1 and A.stride(1) >= max(1, n):
        return A, A.stride(1)
    t = A.t().contiguous().t()
    return t, max(1, n)


def empty_colmajor(n, k, device, dtype=torch.float64):
    return torch.empty((k, n), dtype=dtype, device=device).t()


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # Handles still alive at exit (for instance held by the traceback of an
    # uncaught exception) are destroyed here, while torch and the HIP runtime
    # are intact, instead of during interpreter finalization.  This module is
    # imported after torch, so this runs before torch's own exit handlers.
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


class Handle:
    """A solver handle bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        self._lib = _load()
        stream = stream if stream is not None else torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = self._lib.skew_evd_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise SkewEvdError(st, "skew_evd_create")
        self._h = h
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.skew_evd_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be None at exit)
        if _finalizing():
            return          # the runtime may be gone; _close_all ran before this
        try:
            self.close()
        except Exception:
            pass

    # -- solver --------------------------------------------------------------
    def solve(self, A, nev=None, precision="fp64", band=0, opts=None, info=None, out=None,
              check=True, profile=0):
        """Eigenpairs of the skew-symmetric A (torch float64 CUDA tensor, n x n).

        Returns (lam, Zre, Zim): lam (nev,), Zre/Zim (n, nev) column-major
        views.  Only the strict lower triangle of A is read.
        """
        n = A.shape[0]
        half = (n + 1) // 2
        o = opts if opts is not None else default_opts(precision, band, profile=profile)
        if o.all_pairs:
            nev = n                      # every eigenpair, both signs
        nev = half if nev is None else int(nev)
        Ac, lda = colmajor(A)
        dev = A.device
        if out is None:
            lam = torch.empty(max(nev, 1), dtype=torch.float64, device=dev)
            zr = empty_colmajor(max(n, 1), max(nev, 1), dev)
            zi = empty_colmajor(max(n, 1), max(nev, 1), dev)
        else:
            lam, zr, zi = out
        inf = info if info is not None else Info()
        st = self._lib.skew_evd_ex(self._h, n, ctypes.c_void_p(Ac.data_ptr()), lda, nev,
                                   ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(zr.data_ptr()),
                                   zr.stride(1), ctypes.c_void_p(zi.data_ptr()), zi.stride(1),
                                   ctypes.byref(o), ctypes.byref(inf))
        if check and st not in (OK, WARN_REFINE):
            raise SkewEvdError(st, "skew_evd_ex")
        self.last_status = st
        self.last_info = inf
        return lam[:nev], zr[:n, :nev], zi[:n, :nev]

    def autotune(self, n, precision="fp64"):
        """Band width the autotuner picks for order n (tuned once per size
        class and cached in the handle); returns (band, best ms per solve)."""
        b = ctypes.c_int(0)
        ms = ctypes.c_double(0.0)
        prec = _PREC[precision] if isinstance(precision, str) else int(precision)
        st = self._lib.skew_evd_autotune(self._h, int(n), prec, ctypes.byref(b), ctypes.byref(ms))
        if st != OK:
            raise SkewEvdError(st, "skew_evd_autotune")
        return b.value, ms.value

    def batched_outputs(self, mats, nevs=None):
        """Output buffers for solve_batched(mats, nevs=nevs, out=...)."""
        ns = [int(A.shape[0]) for A in mats]
        nevs = [(x + 1) // 2 for x in ns] if nevs is None else [int(v) for v in nevs]
        dev = mats[0].device if mats else torch.device("cuda")
        return [(torch.empty(max(v, 1), dtype=torch.float64, device=dev),
                 empty_colmajor(max(x, 1), max(v, 1), dev),
                 empty_colmajor(max(x, 1), max(v, 1), dev)) for x, v in zip(ns, nevs)]

    def solve_batched(self, mats, precision="fp64", band=0, autotune=0, nevs=None, reduction=0, out=None,
                      panel_method=0):
        """Solve a list of skew matrices (each n_i x n_i float64 CUDA); returns
        a list of (lam, Zre, Zim), the per-problem status list and the call's
        status.  nevs: eigenpairs per problem (default ceil(n_i / 2)).  out:
        buffers from batched_outputs, reused across calls (a repeated call
        with the same inputs and outputs replays the library's captured
        launch graph)."""
        count = len(mats)
        cols = [colmajor(A) for A in mats]
        ns = [int(A.shape[0]) for A in mats]
        nevs = [(x + 1) // 2 for x in ns] if nevs is None else [int(v) for v in nevs]
        outs = self.batched_outputs(mats, nevs) if out is None else out
        IntA = ctypes.c_int * max(count, 1)
        PtrA = ctypes.c_void_p * max(count, 1)
        n_a = IntA(*ns)
        lda_a = IntA(*[ld for _, ld in cols])
        nev_a = IntA(*nevs)
        A_a = PtrA(*[c.data_ptr() for c, _ in cols])
        l_a = PtrA(*[o[0].data_ptr() for o in outs])
        zr_a = PtrA(*[o[1].data_ptr() for o in outs])
        zi_a = PtrA(*[o[2].data_ptr() for o in outs])
        status = IntA()
        o = default_opts(precision, band, autotune=autotune, reduction=reduction, panel_method=panel_method)
        inf = Info()
        st = self._lib.skew_evd_batched(self._h, count, n_a, A_a, lda_a, nev_a, l_a, zr_a, zi_a,
                                        ctypes.byref(o), ctypes.byref(inf), status)
        self.last_info = inf
        res = [(lm[:v], zr[:x, :v], zi[:x, :v]) for (lm, zr, zi), x, v in zip(outs, ns, nevs)]
        return res, [status[i] for i in range(count)], st

    def bse(self, A, B, nev=None, opts=None, check=True):
        """Bethe-Salpeter eigenpairs of H_BS = [[A, B], [-conj(B), -conj(A)]]
        (A Hermitian, B complex symmetric, complex128 CUDA tensors, m x m).
        Returns (lam, X): the nev smallest positive eigenvalues and the
        eigenvectors x_k (2m x nev complex, x^H S x = 1)."""
        m = A.shape[0]
        nev = m if nev is None else int(nev)
        planes = [colmajor(t)[0] for t in (A.real, A.imag, B.real, B.imag)]
        dev = A.device
        lam = torch.empty(max(nev, 1), dtype=torch.float64, device=dev)
        xr = empty_colmajor(max(2 * m, 1), max(nev, 1), dev)
        xi = empty_colmajor(max(2 * m, 1), max(nev, 1), dev)
        o = opts if opts is not None else default_opts()
        inf = Info()
        st = self._lib.skew_evd_bse(self._h, m, ctypes.c_void_p(planes[0].data_ptr()),
                                    ctypes.c_void_p(planes[1].data_ptr()), planes[0].stride(1),
                                    ctypes.c_void_p(planes[2].data_ptr()), ctypes.c_void_p(planes[3].data_ptr()),
                                    planes[2].stride(1), nev, ctypes.c_void_p(lam.data_ptr()),
                                    ctypes.c_void_p(xr.data_ptr()), ctypes.c_void_p(xi.data_ptr()),
                                    xr.stride(1), ctypes.byref(o), ctypes.byref(inf))
        self.last_status = st
        self.last_info = inf
        if check and st not in (OK, WARN_REFINE):
            raise SkewEvdError(st, "skew_evd_bse")
        return lam[:nev], torch.complex(xr[:2 * m, :nev].contiguous(), xi[:2 * m, :nev].contiguous())

    # -- stage entry points --------------------------------------------------
    def band_reduce(self, A, b):
        n = A.shape[0]
        Ac, lda = colmajor(A)
        band = empty_colmajor(b + 1, max(n, 1), A.device)
        st = self._lib.skew_evd_band_reduce(self._h, n, ctypes.c_void_p(Ac.data_ptr()), lda, b,
                                            ctypes.c_void_p(band.data_ptr()), band.stride(1))
        if st != OK:
            raise SkewEvdError(st, "skew_evd_band_reduce")
        return band[:, :n]

    def tridiagonalize(self, A, b=0):
        n = A.shape[0]
        Ac, lda = colmajor(A)
        alpha = torch.empty(max(n - 1, 1), dtype=torch.float64, device=A.device)
        st = self._lib.skew_evd_tridiagonalize(self._h, n, ctypes.c_void_p(Ac.data_ptr()), lda, b,
                                               ctypes.c_void_p(alpha.data_ptr()))
        if st != OK:
            raise SkewEvdError(st, "skew_evd_tridiagonalize")
        return alpha[:max(n - 1, 0)]

    def tridiag_eig(self, alpha, nev=None):
        n = alpha.numel() + 1
        nev = (n + 1) // 2 if nev is None else int(nev)
        a = alpha.contiguous() if alpha.numel() else torch.zeros(1, dtype=torch.float64,
                                                                  device=alpha.device)
        lam = torch.empty(max(nev, 1), dtype=torch.float64, device=alpha.device)
        Q = empty_colmajor(n, max(nev, 1), alpha.device)
        st = self._lib.skew_evd_tridiag_eig(self._h, n, ctypes.c_void_p(a.data_ptr()), nev,
                                            ctypes.c_void_p(lam.data_ptr()),
                                            ctypes.c_void_p(Q.data_ptr()), Q.stride(1))
        if st != OK:
            raise SkewEvdError(st, "skew_evd_tridiag_eig")
        return lam[:nev], Q[:, :nev]


def noalloc_max_n():
    """SKEW_EVD_NOALLOC_NMAX of the header."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "skew_evd.h")
    return int(re.search(r"#define SKEW_EVD_NOALLOC_NMAX (\d+)", open(hdr).read()).group(1))


def solve_noalloc(A, nev=None, out=None, stream=None):
    """skew_evd_noalloc (the allocation-free entry point): A a float64 CUDA
    tensor of order n <= noalloc_max_n(); returns (status, lam, Zre, Zim).
    With out=(lam, Zre, Zim) (column-major) nothing is allocated here either."""
    n = A.shape[0]
    nev = (n + 1) // 2 if nev is None else int(nev)
    Ac, lda = colmajor(A)
    if out is None:
        dev = A.device
        out = (torch.empty(max(nev, 1), dtype=torch.float64, device=dev),
               empty_colmajor(max(n, 1), max(nev, 1), dev), empty_colmajor(max(n, 1), max(nev, 1), dev))
    lam, zr, zi = out
    stream = stream if stream is not None else torch.cuda.current_stream()
    st = _load().skew_evd_noalloc(n, ctypes.c_void_p(Ac.data_ptr()), lda, nev, ctypes.c_void_p(lam.data_ptr()),
                                  ctypes.c_void_p(zr.data_ptr()), zr.stride(1), ctypes.c_void_p(zi.data_ptr()),
                                  zi.stride(1), ctypes.c_void_p(stream.cuda_stream))
    return st, lam[:nev], zr[:n, :nev], zi[:n, :nev]


_handles = {}


def handle():
    """Per-device default handle on the current stream."""
    dev = torch.cuda.current_device()
    s = torch.cuda.current_stream()
    key = (dev, s.cuda_stream)
    if key not in _handles:
        _handles[key] = Handle(s)
    return _handles[key]


def skew_evd(A, nev=None, precision="fp64", band=0):
    """Convenience: (lam, Z) with Z = Zre + i Zim as a complex128 tensor."""
    lam, zr, zi = handle().solve(A, nev=nev, precision=precision, band=band)
    return lam, torch.complex(zr.contiguous(), zi.contiguous())
