"""GPU tests of the precision form: band reduction and back-transformations in
FP32 on MFMA, then FP64 refinement; results must meet the FP64 tolerances
against the oracle.

Tests that claim the FP32 path assert info.refine_sweeps >= 0 (the refinement
converged; -1 marks a solve handed to the FP64 form).  The cases whose pairs
are closer than the FP32 start resolves are separate tests, named for the
fallback."""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, metrics, solve_np, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


@pytest.mark.parametrize("n", [2, 3, 64, 257, 1000, 2049])
def test_fp32_refine_random(h, n):
    print(f"fp32+refine random n={n}", flush=True)
    A = wl.random_skew(n, 700 + n)
    lam, Z = solve_np(h, A, precision="fp32")
    inf = h.last_info
    lref, _ = oracle.skew_evd(A)
    nA = lref.max()
    err = np.max(np.abs(lam - lref)) / nA
    res, orth, _ = metrics(A, lam, Z, nA)
    print(f"  sweeps={inf.refine_sweeps} resid_est={inf.refine_residual:.1e} err={err:.1e} "
          f"res={res:.1e} orth={orth:.1e}", flush=True)
    assert h.last_status == 0
    assert inf.refine_sweeps >= 0, "the precision form fell back to the FP64 form"
    assert err <= TOL_EIG and res <= TOL_RES and orth <= TOL_ORTH


def test_fp32_refine_prescribed_separated(h):
    """A known spectrum on an even grid in [1, 10] (gaps >= 4.4e-3 at n = 1024):
    the FP32 start separates every pair and the refinement converges."""
    n = 1024
    m = n // 2
    rng = np.random.default_rng(21)
    l = 1.0 + 9.0 * (np.arange(m) + 0.5 + 0.25 * rng.uniform(-1, 1, m)) / m
    A, l = wl.prescribed_large(n, 22, l=l)
    lam, Z = solve_np(h, A, precision="fp32")
    sweeps = h.last_info.refine_sweeps
    assert np.max(np.abs(lam - l)) <= TOL_EIG * l.max()
    res, orth, _ = metrics(A, lam, Z, l.max())
    print(f"  prescribed (separated) res={res:.1e} orth={orth:.1e} sweeps={sweeps}", flush=True)
    assert res <= TOL_RES and orth <= TOL_ORTH
    assert sweeps >= 0, "the precision form fell back to the FP64 form"


def test_fp32_refine_prescribed_close_pairs_fallback(h):
    """Log-uniform l_k in [1e-3, 10] (n = 1024): some pairs are closer than the
    FP32 start resolves, so the solve is handed to the FP64 form
    (refine_sweeps = -1) and still meets the FP64 tolerances."""
    n = 1024
    A, l, Q = wl.prescribed(n, 2)
    lam, Z = solve_np(h, A, precision="fp32")
    sweeps = h.last_info.refine_sweeps
    assert np.max(np.abs(lam - l)) <= TOL_EIG * l.max()
    res, orth, _ = metrics(A, lam, Z, l.max())
    print(f"  prescribed (close pairs) res={res:.1e} orth={orth:.1e} sweeps={sweeps}", flush=True)
    assert res <= TOL_RES and orth <= TOL_ORTH
    assert sweeps == -1


def test_fp32_no_fallback_returns_warn_refine(h):
    """With no_fp64_fallback = 1 and no refinement sweep allowed, the solve
    returns WARN_REFINE and the unrefined FP32 eigenpairs (accurate to the FP32
    level only)."""
    from paper_1912_04062_amd import skewevd
    n = 700
    A = wl.random_skew(n, 31)
    o = skewevd.default_opts("fp32", max_refine_sweeps=0, no_fp64_fallback=1)
    lam, zr, zi = h.solve(to_dev(A), opts=o)
    assert h.last_status == skewevd.WARN_REFINE
    assert h.last_info.refine_sweeps == 0
    lam = lam.cpu().numpy()
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    lref, _ = oracle.skew_evd(A)
    err = np.max(np.abs(lam - lref)) / lref.max()
    res, orth, _ = metrics(A, lam, Z, lref.max())
    print(f"  unrefined err={err:.1e} res={res:.1e} orth={orth:.1e}", flush=True)
    # the eigenvalues come from the first FP64 measurement of the refinement
    # (Rayleigh quotients, accurate to the square of the vectors' error)
    assert err <= 1e-8 and res <= 1e-6 and orth <= 1e-6
    assert res > 1e-13 and orth > 1e-13      # the FP32 vectors, not an FP64 result


def test_fp32_odd_null(h):
    n = 301
    A = wl.random_skew(n, 5)
    lam, Z = solve_np(h, A, precision="fp32")
    assert h.last_info.refine_sweeps >= 0
    assert lam[0] == 0.0
    assert np.all(Z[:, 0].imag == 0.0)
    assert np.linalg.norm(A @ Z[:, 0].real) <= 1e-13 * lam.max() * np.sqrt(n)


def test_fp32_refine_uneven_batch_matrices(h):
    """Every matrix of the uneven batch (512 orders in 64..1024, seed 5) solved
    one by one in the precision form.  Some of them hold pairs closer than the
    FP32 start resolves; their refinement must either converge or hand the
    problem to the FP64 form: every result meets the FP64 tolerances."""
    import torch
    sizes, mats = wl.batch(512, 5)
    print(f"fp32+refine on {len(sizes)} batch matrices, n in [{min(sizes)}, {max(sizes)}]", flush=True)
    worst_r, worst_o, fallbacks = 0.0, 0.0, 0
    for i, A in enumerate(mats):
        n = A.shape[0]
        Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
        lam, zr, zi = h.solve(Ad, precision="fp32")
        fallbacks += h.last_info.refine_sweeps < 0
        Af = torch.tril(Ad.contiguous(), -1)
        Af = Af - Af.t()
        Z = torch.complex(zr.contiguous(), zi.contiguous())
        R = torch.complex(Af, torch.zeros_like(Af)) @ Z - Z * (1j * lam)[None, :]
        nA = lam.max().item()
        r = torch.linalg.norm(R).item() / (n * nA)
        G = Z.conj().t() @ Z
        G.diagonal().sub_(1.0)
        o = torch.linalg.norm(G).item() / n
        assert r <= TOL_RES and o <= TOL_ORTH, (i, n, r, o, h.last_info.refine_sweeps)
        worst_r, worst_o = max(worst_r, r), max(worst_o, o)
        if i % 64 == 0:                              # oracle sample
            lref, _ = oracle.skew_evd(A)
            assert np.max(np.abs(lam.cpu().numpy() - lref)) <= TOL_EIG * lref.max()
    print(f"  worst res={worst_r:.2e} orth={worst_o:.2e}, FP64 fallbacks {fallbacks}", flush=True)
