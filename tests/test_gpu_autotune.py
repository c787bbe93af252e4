"""GPU tests of the band-width autotuner and the autotuned batched form.

The tuner only chooses among supported band widths, so its results are checked
like any other solve: against the oracle (eigenvalues within 1e-12 ||A||) and
by residual and orthogonality (1e-13), and bitwise against a single solve with
the same tuned configuration (band width and panel method: same kernels, same
tiles).
"""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, metrics, to_dev

pytestmark = pytest.mark.gpu

CAND = (16, 32, 64)


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


def test_autotune_picks_a_supported_band_and_caches_it(h):
    print("autotune n=200 fp64", flush=True)
    b, ms = h.autotune(200)
    assert b in CAND and ms > 0.0
    # same size class (129..256): cached, identical answer
    assert h.autotune(250) == (b, ms)
    b2, _ = h.autotune(60)
    assert b2 in CAND


def test_unsupported_band_is_an_argument_error(h):
    # only 8, 16, 32 and 64 have panel kernels: anything else is rejected
    # before any launch (argument 11, the options)
    A = wl.random_skew(100, 3)
    for b in (24, 48, 12, 128):
        h.solve(to_dev(A), band=b, check=False)
        assert h.last_status == -11, b


def test_ex_autotune_takes_the_tuned_band(h):
    import torch
    from paper_1912_04062_amd import skewevd
    n = 300
    A = wl.random_skew(n, 31)
    print(f"solve n={n} autotune", flush=True)
    lam, zr, zi = h.solve(to_dev(A), opts=skewevd.default_opts(autotune=1))
    torch.cuda.synchronize()
    b, _ = h.autotune(n)
    assert h.last_info.band == b
    lam = lam.cpu().numpy()
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    lref, _ = oracle.skew_evd(A)
    assert np.max(np.abs(lam - lref)) <= TOL_EIG * lref.max()
    res, orth, _ = metrics(A, lam, Z, lref.max())
    assert res <= TOL_RES and orth <= TOL_ORTH


def test_batched_autotuned_matches_oracle_and_single_solves(h):
    import torch
    from paper_1912_04062_amd import skewevd
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(64, 512, size=10, endpoint=True)]
    sizes += [65, 129]            # odd orders: the exact zero eigenvalue
    mats = [wl.random_skew(x, 500 + i) for i, x in enumerate(sizes)]
    print(f"batched autotune sizes={sizes}", flush=True)
    res, status, st = h.solve_batched([to_dev(A) for A in mats], autotune=1)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in status)
    for A, (lam, zr, zi) in zip(mats, res):
        n = A.shape[0]
        b, _ = h.autotune(n)
        lam = lam.cpu().numpy()
        zr = zr.cpu().numpy()
        zi = zi.cpu().numpy()
        # a single solve with the same tuned configuration (band and panel method)
        l1, z1r, z1i = h.solve(to_dev(A), opts=skewevd.default_opts(autotune=1))
        assert h.last_info.band == b
        assert np.array_equal(lam, l1.cpu().numpy())
        assert np.array_equal(zr, z1r.cpu().numpy()) and np.array_equal(zi, z1i.cpu().numpy())
        lref, _ = oracle.skew_evd(A)
        assert np.max(np.abs(lam - lref)) <= TOL_EIG * lref.max()
        if n % 2:
            assert lam[0] == 0.0
        res_, orth, _ = metrics(A, lam, zr + 1j * zi, lref.max())
        assert res_ <= TOL_RES and orth <= TOL_ORTH, (n, b, res_, orth)
