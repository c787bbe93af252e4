"""GPU parity tests: the HIP path (through the C-ABI) against the oracle.

Tolerances (FP64, from the parity contract): eigenvalue error <= 1e-12 ||A||,
residual ||AZ - Z diag(i lam)||_F / (n ||A||) <= 1e-13, orthogonality
||Z^H Z - I||_F / n <= 1e-13.  Eigenvectors are compared phase-invariantly
(the phase of each z_k is not unique) for well-separated eigenvalues; near-
degenerate ones are checked through residual and orthogonality only.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import (TOL_EIG, TOL_ORTH, TOL_RES, band_to_dense, metrics, phase_match,
                      solve_np, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


def _log(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# Stage level
@pytest.mark.parametrize("n,b", [(40, 8), (300, 16), (700, 32), (1100, 64), (129, 64)])
def test_band_reduce(h, n, b):
    _log(f"band_reduce n={n} b={b}")
    A = wl.random_skew(n, 100 + n)
    band = h.band_reduce(to_dev(A), b).cpu().numpy()
    B = band_to_dense(band, n, b)
    assert abs(np.linalg.norm(B) - np.linalg.norm(A)) <= 1e-13 * np.linalg.norm(A)
    la, _ = oracle.skew_evd(A)
    lb, _ = oracle.skew_evd(B)
    assert np.max(np.abs(la - lb)) <= TOL_EIG * la.max()


@pytest.mark.parametrize("n,b", [(10, 8), (65, 16), (500, 32), (1030, 64)])
def test_tridiagonalize(h, n, b):
    _log(f"tridiagonalize n={n} b={b}")
    A = wl.random_skew(n, 200 + n)
    alpha = h.tridiagonalize(to_dev(A), b).cpu().numpy()
    fro2 = np.sum(A * A)
    assert abs(2 * np.sum(alpha ** 2) - fro2) <= 1e-12 * fro2
    la, _ = oracle.skew_evd(A)
    lt = oracle.tridiag_eigvals(alpha, n // 2, (n + 1) // 2)
    assert np.max(np.abs(la - np.maximum(lt, 0))) <= TOL_EIG * la.max()


@pytest.mark.parametrize("n", [2, 7, 64, 501, 2000])
def test_tridiag_eig_random(h, n):
    import torch
    _log(f"tridiag_eig random n={n}")
    rng = np.random.default_rng(300 + n)
    alpha = rng.standard_normal(n - 1)
    lam, Q = h.tridiag_eig(torch.from_numpy(alpha).cuda())
    lam, Q = lam.cpu().numpy(), Q.cpu().numpy()
    ref = oracle.tridiag_eigvals(alpha, n // 2, (n + 1) // 2)
    T = np.diag(alpha, 1) + np.diag(alpha, -1)
    nT = np.abs(np.linalg.eigvalsh(T)).max()
    assert np.max(np.abs(lam - ref)) <= TOL_EIG * nT
    assert np.linalg.norm(T @ Q - Q * lam[None, :]) / (n * nT) <= TOL_RES
    assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) / n <= TOL_ORTH


@pytest.mark.parametrize("n", [100, 513])
def test_tridiag_eig_clement(h, n):
    import torch
    _log(f"tridiag_eig clement n={n}")
    j = np.arange(1, n)
    alpha = np.sqrt(j * (n - j).astype(float))
    lam, Q = h.tridiag_eig(torch.from_numpy(alpha).cuda())
    lam = lam.cpu().numpy()
    exact = np.sort(np.array([n - 1 - 2 * k for k in range(n)], float))[n // 2:]
    assert np.max(np.abs(lam - exact)) <= TOL_EIG * (n - 1)


# ---------------------------------------------------------------------------
# Whole solver
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 100, 257, 512, 513, 1000])
def test_solve_random(h, n):
    _log(f"solve random n={n}")
    A = wl.random_skew(n, 1 if n == 512 else 400 + n)
    b = 32 if n == 512 else 0
    lam, Z = solve_np(h, A, band=b)
    lref, Zref = oracle.skew_evd(A)
    nA = max(lref.max(), 1e-300) if n > 1 else 1.0
    assert np.max(np.abs(lam - lref)) <= TOL_EIG * nA
    if n > 1:
        res, orth, _ = metrics(A, lam, Z, nA)
        _log(f"  res={res:.2e} orth={orth:.2e}")
        assert res <= TOL_RES and orth <= TOL_ORTH
        ok, worst = phase_match(Z, Zref, lref, 1e-4 * nA, 1e-10)
        assert ok, worst
    else:
        assert abs(abs(Z[0, 0]) - 1.0) < 1e-15


@pytest.mark.parametrize("n", [1024, 2049])
def test_solve_prescribed(h, n):
    _log(f"solve prescribed n={n}")
    A, l, Q = wl.prescribed(n, 2)
    lam, Z = solve_np(h, A)
    ref = np.concatenate([[0.0] if n % 2 else [], l])
    assert np.max(np.abs(lam - ref)) <= TOL_EIG * l.max()
    res, orth, _ = metrics(A, lam, Z, l.max())
    _log(f"  res={res:.2e} orth={orth:.2e}")
    assert res <= TOL_RES and orth <= TOL_ORTH
    off = 1 if n % 2 else 0
    Zref = np.stack([(Q[:, 2 * p] + 1j * Q[:, 2 * p + 1]) / np.sqrt(2) for p in range(len(l))], 1)
    ok, worst = phase_match(Z[:, off:], Zref, l, 1e-4 * l.max(), 1e-10)
    assert ok, worst


def test_solve_bse(h):
    m = 400
    _log(f"solve bse m={m}")
    K, Ab, Bb = wl.bse_shaped(m, 3)
    lam, Z = solve_np(h, K)
    Lp = np.linalg.cholesky(Ab + Bb)
    ref = np.sqrt(np.sort(np.linalg.eigvalsh(Lp.T @ (Ab - Bb) @ Lp)))
    assert np.max(np.abs(lam - ref)) <= TOL_EIG * ref.max()
    res, orth, _ = metrics(K, lam, Z, ref.max())
    assert res <= TOL_RES and orth <= TOL_ORTH


@pytest.mark.parametrize("n", [3, 101, 257])
def test_odd_null_vector(h, n):
    _log(f"odd null n={n}")
    A = wl.random_skew(n, 5)
    lam, Z = solve_np(h, A)
    assert lam[0] == 0.0
    assert np.all(Z[:, 0].imag == 0.0)
    assert np.linalg.norm(A @ Z[:, 0].real) <= 1e-13 * lam.max() * np.sqrt(n)


@pytest.mark.parametrize("l", [2.5, -0.75])
def test_n2(h, l):
    A = np.array([[0.0, -l], [l, 0.0]], order="F")
    lam, Z = solve_np(h, A)
    assert abs(lam[0] - abs(l)) <= 1e-15 * abs(l)
    ref = np.array([1.0, -1j * np.sign(l)]) / np.sqrt(2.0)
    assert abs(abs(np.vdot(ref, Z[:, 0])) - 1) < 1e-14


@pytest.mark.parametrize("n", [6, 7, 130])
def test_zero_matrix(h, n):
    A = np.zeros((n, n), order="F")
    lam, Z = solve_np(h, A)
    assert np.all(lam == 0.0)                # ||A|| = 0: the tolerance is 0
    assert np.linalg.norm(Z.conj().T @ Z - np.eye(Z.shape[1])) / n <= TOL_ORTH


def test_partial_nev(h):
    n = 300
    A = wl.random_skew(n, 12)
    lam, Z = solve_np(h, A, nev=37)
    lref, _ = oracle.skew_evd(A, nev=37)
    assert lam.shape == (37,)
    assert np.max(np.abs(lam - lref)) <= TOL_EIG * lref.max()
    R = A @ Z - Z * (1j * lam)[None, :]
    assert np.linalg.norm(R) / (n * lref.max()) <= TOL_RES


def test_nonfinite(h):
    from paper_1912_04062_amd import skewevd
    A = wl.random_skew(50, 1)
    A[30, 10] = np.nan
    with pytest.raises(skewevd.SkewEvdError) as e:
        h.solve(to_dev(A))
    assert e.value.status == skewevd.ERR_NONFINITE
    A[30, 10] = 0.0
    A[10, 30] = np.inf          # upper triangle is never read
    lam, _, _ = h.solve(to_dev(A))
    assert np.isfinite(lam.cpu().numpy()).all()


def test_batched_matches_single(h):
    rng = np.random.default_rng(9)
    sizes = [int(x) for x in rng.integers(64, 300, size=6)]
    mats = [wl.random_skew(x, 900 + i) for i, x in enumerate(sizes)]
    res, status, st = h.solve_batched([to_dev(A) for A in mats])
    assert st == 0 and all(s == 0 for s in status)
    for A, (lam, zr, zi) in zip(mats, res):
        l1, z1r, z1i = h.solve(to_dev(A))
        assert np.array_equal(lam.cpu().numpy(), l1.cpu().numpy())
        assert np.array_equal(zr.cpu().numpy(), z1r.cpu().numpy())
        lref, _ = oracle.skew_evd(A)
        assert np.max(np.abs(lam.cpu().numpy() - lref)) <= TOL_EIG * lref.max()


@pytest.mark.parametrize("n,b", [(130, 64), (300, 64), (701, 64), (1000, 64), (700, 16), (1000, 32)])
def test_solve_band_widths(h, n, b):
    """Every band width path of the back-transformations, with ragged tails."""
    _log(f"solve n={n} band={b}")
    A = wl.random_skew(n, 1300 + n + b)
    lam, Z = solve_np(h, A, band=b)
    lref, Zref = oracle.skew_evd(A)
    nA = lref.max()
    assert np.max(np.abs(lam - lref)) <= TOL_EIG * nA
    res, orth, _ = metrics(A, lam, Z, nA)
    _log(f"  res={res:.2e} orth={orth:.2e}")
    assert res <= TOL_RES and orth <= TOL_ORTH
    ok, worst = phase_match(Z, Zref, lref, 1e-4 * nA, 1e-10)
    assert ok, worst
