"""Oracle for the skew-symmetric eigensolver — TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 host implementation (``skew_oracle.c``) of Algorithm 1 of
Penke et al., "High Performance Solution of Skew-symmetric Eigenvalue Problems
with Applications in Solving the Bethe-Salpeter Eigenvalue Problem": one-stage
Householder tridiagonalization with the skew rank-2 update (Section 2.3.1),
the symmetrization of Lemma 1, Sturm bisection plus inverse iteration on the
symmetric tridiagonal (the BSEPACK tridiagonal method, Section 3), the
diagonal back-transformation by D (Algorithm 1, step 3) and the Householder
back-transformation (step 4), applied to real and imaginary parts apart.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skew_oracle.c")
_LIB = os.path.join(_HERE, "libskew_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-fno-fast-math", "-o", _LIB, _SRC, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.check_call(cmd)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_skew_evd.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                    dp, dp, dp, ctypes.c_int]
    lib.oracle_skew_evd.restype = ctypes.c_int
    lib.oracle_skew_tridiag.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp,
                                        ctypes.c_int, dp]
    lib.oracle_skew_tridiag.restype = ctypes.c_int
    lib.oracle_sturm_count.argtypes = [ctypes.c_int, dp, ctypes.c_double]
    lib.oracle_sturm_count.restype = ctypes.c_int
    lib.oracle_tridiag_eigvals.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_tridiag_eigvals.restype = ctypes.c_int
    lib.oracle_tridiag_eigvecs.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp,
                                           ctypes.c_int, ctypes.c_uint64]
    lib.oracle_tridiag_eigvecs.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    pass


def skew_evd(A, nev=None):
    """Eigenpairs of the skew-symmetric A (only its strict lower triangle is read).

    Returns (lam, Z) with lam ascending (the nev smallest of the ceil(n/2)
    values lambda >= 0) and Z complex (n x nev), A Z = Z diag(+i lam).
    """
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    half = (n + 1) // 2
    nev = half if nev is None else int(nev)
    lam = np.zeros(max(nev, 1))
    zr = np.zeros((max(n, 1), max(nev, 1)), order="F")
    zi = np.zeros((max(n, 1), max(nev, 1)), order="F")
    Abuf = A if n > 0 else np.zeros((1, 1), order="F")
    st = _load().oracle_skew_evd(n, _ptr(Abuf), max(n, 1), nev, _ptr(lam), _ptr(zr),
                                 _ptr(zi), max(n, 1))
    if st != 0:
        raise OracleError(f"oracle_skew_evd returned status {st}")
    return lam[:nev].copy(), (zr[:n, :nev] + 1j * zi[:n, :nev])


def skew_evd_status(A, nev):
    """Status code only (argument validation / non-finite checks)."""
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    lam = np.zeros(max(nev, 1))
    zr = np.zeros((max(n, 1), max(nev, 1)), order="F")
    zi = np.zeros_like(zr)
    Abuf = A if n > 0 else np.zeros((1, 1), order="F")
    return _load().oracle_skew_evd(n, _ptr(Abuf), max(n, 1), nev, _ptr(lam), _ptr(zr),
                                   _ptr(zi), max(n, 1))


def tridiagonalize(A):
    """Step 1 only: (alpha, V, tau) with alpha the super-diagonal of A_trd."""
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    alpha = np.zeros(max(n, 1))
    V = np.zeros((max(n, 1), max(n, 1)), order="F")
    tau = np.zeros(max(n, 1))
    st = _load().oracle_skew_tridiag(n, _ptr(A), max(n, 1), _ptr(alpha), _ptr(V), max(n, 1),
                                     _ptr(tau))
    if st != 0:
        raise OracleError(f"oracle_skew_tridiag returned status {st}")
    return alpha[:max(n - 1, 0)].copy(), V[:n, :n].copy(), tau[:n].copy()


def sturm_count(alpha, x):
    """Number of eigenvalues of tridiag(alpha, 0, alpha) strictly below x."""
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    n = alpha.size + 1
    buf = alpha if alpha.size else np.zeros(1)
    return _load().oracle_sturm_count(n, _ptr(buf), float(x))


def tridiag_eigvals(alpha, first, count):
    """Eigenvalues first..first+count-1 (ascending) of tridiag(alpha, 0, alpha)."""
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    n = alpha.size + 1
    w = np.zeros(max(count, 1))
    buf = alpha if alpha.size else np.zeros(1)
    st = _load().oracle_tridiag_eigvals(n, _ptr(buf), int(first), int(count), _ptr(w))
    if st != 0:
        raise OracleError(f"oracle_tridiag_eigvals returned status {st}")
    return w[:count].copy()


def tridiag_eigvecs(alpha, w, seed=0x5EED):
    """Eigenvectors of tridiag(alpha, 0, alpha) for the ascending values w."""
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    n = alpha.size + 1
    Q = np.zeros((n, max(w.size, 1)), order="F")
    buf = alpha if alpha.size else np.zeros(1)
    st = _load().oracle_tridiag_eigvecs(n, _ptr(buf), w.size, _ptr(w), _ptr(Q), n, seed)
    if st != 0:
        raise OracleError(f"oracle_tridiag_eigvecs returned status {st}")
    return Q[:, :w.size].copy()


def bse_evd(A, B, nev=None):
    """The Bethe-Salpeter route of Section 3 (the four BSEPACK steps), as plain
    numpy steps around the skew-symmetric oracle above.

    A (m x m, Hermitian) and B (m x m, complex symmetric) define
    H_BS = [[A, B], [-conj(B), -conj(A)]] (Eq. BSmatrix), assumed definite
    ([[A, B], [conj(B), conj(A)]] > 0).  Steps:
      1. M = [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]] (Eq. SymmetricM, M = JH);
      2. Cholesky M = L L^T;
      3. eigenpairs K z = i lambda z of the skew-symmetric K = L^T J L,
         J = [[0, I], [-I, 0]] (the skew oracle);
      4. back-transformation (Theorem 2 and the Cholesky factor): with
         H = J^T M, H L^{-T} z = -i lambda L^{-T} z, so x = Q L^{-T} z,
         Q = [[I, -iI], [I, iI]] / sqrt(2), satisfies H_BS x = lambda x.
    x is scaled to the BSE normalization x^H S x = 1, S = diag(I, -I)
    (unscaled, x^H S x = 1 / lambda for ||z|| = 1).
    Returns (lam, X): the nev smallest positive eigenvalues of H_BS ascending
    and X (2m x nev complex)."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    m = A.shape[0]
    n = 2 * m
    nev = m if nev is None else int(nev)
    M = np.block([[(A + B).real, (A - B).imag], [-(A + B).imag, (A - B).real]])
    L = np.linalg.cholesky(M)
    J = np.block([[np.zeros((m, m)), np.eye(m)], [-np.eye(m), np.zeros((m, m))]])
    K = L.T @ J @ L
    lam, Z = skew_evd(np.asfortranarray(K), nev)
    W = np.linalg.solve(L.T, Z)                       # L^{-T} z (a triangular solve)
    X = np.vstack([W[:m] - 1j * W[m:], W[:m] + 1j * W[m:]]) / np.sqrt(2.0)
    return lam, X * np.sqrt(lam)[None, :]


def num_threads():
    return _load().oracle_num_threads()
