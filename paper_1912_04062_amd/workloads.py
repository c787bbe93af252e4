"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles test matrices; it holds
none of the eigensolver's arithmetic.  It is shared by the tests, the smoke
check and the benchmark (GPU side and oracle side alike).

* ``random_skew``   - dense A = (B - B^T)/2 with B iid N(0, 1): the random
                       double-precision skew-symmetric matrices of the paper's
                       ELPA benchmarks (Section 4.1).
* ``prescribed``    - A = Q blockdiag([[0, l_k], [-l_k, 0]]) Q^T with Q Haar
                       orthogonal and l_k log-uniform: known spectrum +-i*l_k
                       and known eigenvectors (q_2k + i q_2k+1)/sqrt(2).
* ``bse_shaped``    - the skew matrix L^T J L of the Bethe-Salpeter route
                       (Section 3: M = J H > 0, Cholesky M = L L^T), built from
                       a synthetic real M = [[A, B], [B, A]].  It stands in for
                       the hexagonal boron nitride Hamiltonian of Section 4.2,
                       which is not available.
* ``prescribed_large`` - a known spectrum at large n, cheap to form:
                       A = Q1 P Q2 S Q2 P^T Q1 with symmetric orthogonal block
                       reflectors Q_i = I - 2 U_i U_i^T (U_i: n x k, orthonormal
                       columns) and a random permutation P.
* ``tridiag_blocks`` - an already tridiagonal skew matrix that splits into
                       identical blocks (every eigenvalue of a block is repeated
                       once per block).
* ``bse_complex``   - complex Hermitian A and complex symmetric B of a definite
                       Bethe-Salpeter Hamiltonian [[A, B], [-conj(B), -conj(A)]].
* ``batch_sizes``   - matrix orders for a batch of uneven problems.

All matrices are returned as Fortran-ordered (column-major) float64 arrays.
"""
import numpy as np


def random_skew(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    A = np.asfortranarray((B - B.T) * 0.5)
    return A


def haar_orthogonal(n, rng):
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of R's diagonal moved into Q (Mezzadri 2007)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def prescribed(n, seed, lo=1e-3, hi=10.0):
    """Skew matrix with prescribed spectrum.

    Returns (A, l, Q): l (ascending, length n//2) are the positive eigenvalue
    magnitudes, Q the orthogonal basis; for odd n the last column of Q spans
    the null space.  The eigenvector of +i*l[k] is (Q[:, 2p] + i Q[:, 2p+1])/sqrt(2)
    where p is the block index of l[k] (blocks are laid out in ascending order).
    """
    rng = np.random.default_rng(seed)
    Q = haar_orthogonal(n, rng)
    m = n // 2
    l = np.sort(10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=m))
    S = np.zeros((n, n))
    for p in range(m):
        S[2 * p, 2 * p + 1] = l[p]
        S[2 * p + 1, 2 * p] = -l[p]
    A = Q @ S @ Q.T
    A = np.asfortranarray((A - A.T) * 0.5)
    return A, l, Q


def _reflect(B, U):
    """(I - 2 U U^T) B (I - 2 U U^T) for U with orthonormal columns, in place."""
    C = U.T @ B                      # k x n
    B -= 2.0 * (U @ C)
    D = B @ U                        # n x k (after the left product)
    B -= 2.0 * (D @ U.T)
    return B


def prescribed_large(n, seed, l=None, k=64, lo=1e-3, hi=10.0):
    """Skew matrix of even order n with the prescribed spectrum +-i*l.

    l: the n/2 magnitudes (ascending), or None for log-uniform in [lo, hi].
    A = Q1 P Q2 S Q2 P^T Q1, S = blockdiag([[0, l_p], [-l_p, 0]]); forming it
    costs a few n x n x k products, so it serves at n = 16384.  Returns (A, l)
    with l ascending."""
    assert n % 2 == 0
    rng = np.random.default_rng(seed)
    m = n // 2
    if l is None:
        l = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=m)
    l = np.sort(np.asarray(l, dtype=np.float64))
    B = np.zeros((n, n))
    idx = np.arange(m)
    B[2 * idx, 2 * idx + 1] = l
    B[2 * idx + 1, 2 * idx] = -l
    U2, _ = np.linalg.qr(rng.standard_normal((n, k)))
    _reflect(B, U2)
    perm = rng.permutation(n)
    B = B[perm][:, perm]
    U1, _ = np.linalg.qr(rng.standard_normal((n, k)))
    _reflect(B, U1)
    A = np.asfortranarray((B - B.T) * 0.5)
    return A, l


def tridiag_blocks(n, pattern):
    """Tridiagonal skew A (A[j+1, j] = s_j, A[j, j+1] = -s_j) whose
    sub-diagonal repeats `pattern` followed by a 0, so that A splits into
    identical blocks of order len(pattern) + 1 (n a multiple of that)."""
    q = len(pattern) + 1
    assert n % q == 0
    s = np.tile(np.concatenate([np.asarray(pattern, float), [0.0]]), n // q)[: n - 1]
    A = np.zeros((n, n), order="F")
    j = np.arange(n - 1)
    A[j + 1, j] = s
    A[j, j + 1] = -s
    return A


def bse_blocks(m, seed, rank=64):
    """Real symmetric blocks A = diag(d) + V V^T/m, B = 0.1 W W^T/m."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(1.0, 10.0, size=m)
    V = rng.standard_normal((m, rank))
    W = rng.standard_normal((m, rank))
    Ab = np.diag(d) + V @ V.T / m
    Bb = 0.1 * (W @ W.T) / m
    return Ab, Bb


def bse_shaped(m, seed, rank=64):
    """K = L^T J L with M = [[A, B], [B, A]] = L L^T (n = 2m).

    Returns (K, Ab, Bb).  The spectrum of K is +-i*sqrt(eig((A+B)(A-B))).
    """
    Ab, Bb = bse_blocks(m, seed, rank)
    M = np.block([[Ab, Bb], [Bb, Ab]])
    L = np.linalg.cholesky(M)
    n = 2 * m
    # J L = [[L_bottom], [-L_top]]  (J = [[0, I], [-I, 0]])
    JL = np.vstack([L[m:, :], -L[:m, :]])
    K = L.T @ JL
    K = np.asfortranarray((K - K.T) * 0.5)
    return K, Ab, Bb


def bse_complex(m, seed, rank=64):
    """Complex Bethe-Salpeter blocks: A Hermitian, B complex symmetric, with
    [[A, B], [conj(B), conj(A)]] > 0 (the definite case of Section 3).
    A = diag(d) + V V^H / m (d ~ U[1, 10], V m x rank complex Gaussian),
    B = 0.1 W W^T / m (W m x rank complex Gaussian): ||B|| is small against
    A >= 1, so the block matrix is positive definite.  Returns (A, B)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(1.0, 10.0, size=m)
    V = (rng.standard_normal((m, rank)) + 1j * rng.standard_normal((m, rank))) / np.sqrt(2.0)
    W = (rng.standard_normal((m, rank)) + 1j * rng.standard_normal((m, rank))) / np.sqrt(2.0)
    A = np.diag(d).astype(np.complex128) + V @ V.conj().T / m
    A = (A + A.conj().T) * 0.5
    B = 0.1 * (W @ W.T) / m
    B = (B + B.T) * 0.5
    return np.asfortranarray(A), np.asfortranarray(B)


def batch_sizes(count, seed, lo=64, hi=1024):
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi, size=count, endpoint=True)]


def batch(count, seed, lo=64, hi=1024):
    """A batch of random skew matrices of uneven order (one generator stream)."""
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(lo, hi, size=count, endpoint=True)]
    mats = []
    for n in sizes:
        B = rng.standard_normal((n, n))
        mats.append(np.asfortranarray((B - B.T) * 0.5))
    return sizes, mats
