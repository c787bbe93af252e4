"""GPU tests of the precision form: band reduction and back-transformations in
FP32 on MFMA, then FP64 refinement; results must meet the FP64 tolerances
against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, metrics, solve_np

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
    assert err <= TOL_EIG and res <= TOL_RES and orth <= TOL_ORTH


def test_fp32_refine_prescribed(h):
    n = 1024
    A, l, Q = wl.prescribed(n, 2)
    lam, Z = solve_np(h, A, precision="fp32")
    assert np.max(np.abs(lam - l)) <= TOL_EIG * l.max()
    res, orth, _ = metrics(A, lam, Z, l.max())
    print(f"  prescribed res={res:.1e} orth={orth:.1e} sweeps={h.last_info.refine_sweeps}", flush=True)
    assert res <= TOL_RES and orth <= TOL_ORTH


def test_fp32_odd_null(h):
    n = 301
    A = wl.random_skew(n, 5)
    lam, Z = solve_np(h, A, precision="fp32")
    assert lam[0] == 0.0
    assert np.all(Z[:, 0].imag == 0.0)
    assert np.linalg.norm(A @ Z[:, 0].real) <= 1e-13 * lam.max() * np.sqrt(n)
