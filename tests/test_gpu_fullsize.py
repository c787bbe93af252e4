"""Full-size GPU checks at the workload sizes (in the same launch configuration
the benchmark times): properties that hold at any size, and exact pins where
the input has a known spectrum.

Every case asserts, with FP64 products on the GPU (torch, independent of the
library):
  * the global residual ||AZ - Z diag(i lam)||_F / (n ||A||) <= 1e-13 and
    orthogonality ||Z^H Z - I||_F / n <= 1e-13;
  * the per-column residual max_k ||A z_k - i lam_k z_k||_2 <= 1e-12 ||A||:
    A is normal, so each lam_k then lies within 1e-12 ||A|| of an eigenvalue
    of A (Bauer-Fike), and with orthonormal z_k no eigenvalue is returned
    twice for a simple one.
Pins of the eigenvalues themselves:
* C4 n = 16384 random (both forms): the trace identities sum lambda^2 =
  ||A||_F^2 / 2 and sum lambda^4 = ||A^2||_F^2 / 2 (they fail if an eigenvalue
  is missing, duplicated or wrong).
* n = 16384 prescribed spectrum (both forms): every eigenvalue element-wise
  against the exact l_k, <= 1e-12 ||A||.
* C2 n = 8192 prescribed spectrum: eigenvalues against the exact l_k.
* C3 n = 10000 BSE-shaped: eigenvalues against sqrt(eig(L+^T (A-B) L+)).
* C5 batch of 512 uneven matrices: residual/orthogonality of every matrix,
  eigenvalues of a sample against the oracle.
The precision-form cases assert that the refinement converged
(info.refine_sweeps >= 0), i.e. that no FP64 re-solve produced the result.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, dev_checks, fmt, to_dev

pytestmark = pytest.mark.gpu

TOL_COLRES = 1e-12


@pytest.fixture(scope="module")
def h():
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


def _assert_pairs(c):
    assert c["res"] <= TOL_RES and c["orth"] <= TOL_ORTH, c
    assert c["colres"] <= TOL_COLRES, c


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c4_random_16384(h, precision):
    import torch
    n = 16384
    print(f"C4 n={n} {precision}", flush=True)
    Ad = to_dev(wl.random_skew(n, 4))
    lam, zr, zi = h.solve(Ad, precision=precision)
    torch.cuda.synchronize()
    sweeps = h.last_info.refine_sweeps
    assert lam.numel() == n // 2
    assert bool((lam[1:] >= lam[:-1]).all()) and lam[0].item() >= 0.0
    c = dev_checks(Ad, lam, zr, zi)
    print(f"  {fmt(c)} sweeps={sweeps}", flush=True)
    _assert_pairs(c)
    assert c["tr2"] <= 1e-13 and c["tr4"] <= 1e-12
    if precision == "fp32":
        assert sweeps >= 0, "the precision form fell back to the FP64 form"


def _spaced(m, seed):
    """m magnitudes on an even grid in [1, 10] with jitter of a quarter step:
    gaps of at least half a step (well separated for the FP32 start)."""
    rng = np.random.default_rng(seed)
    return 1.0 + 9.0 * (np.arange(m) + 0.5 + 0.25 * rng.uniform(-1, 1, m)) / m


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_prescribed_16384(h, precision):
    """Element-wise eigenvalues at the headline order against a known spectrum
    (log-uniform in [1e-3, 10] for FP64; an even grid in [1, 10] for the
    precision form, whose FP32 start resolves it)."""
    import torch
    n = 16384
    print(f"prescribed n={n} {precision}", flush=True)
    l = None if precision == "fp64" else _spaced(n // 2, 44)
    A, l = wl.prescribed_large(n, 16, l=l)
    Ad = to_dev(A)
    del A
    lam, zr, zi = h.solve(Ad, precision=precision)
    torch.cuda.synchronize()
    sweeps = h.last_info.refine_sweeps
    err = np.max(np.abs(lam.cpu().numpy() - l)) / l.max()
    c = dev_checks(Ad, lam, zr, zi, nA=l.max())
    print(f"  eig err={err:.2e} {fmt(c)} sweeps={sweeps}", flush=True)
    assert err <= TOL_EIG
    _assert_pairs(c)
    if precision == "fp32":
        assert sweeps >= 0, "the precision form fell back to the FP64 form"


def test_c2_prescribed_8192(h):
    import torch
    n = 8192
    print(f"C2 n={n}", flush=True)
    A, l, _ = wl.prescribed(n, 2)
    Ad = to_dev(A)
    del A
    lam, zr, zi = h.solve(Ad, band=64)
    torch.cuda.synchronize()
    err = np.max(np.abs(lam.cpu().numpy() - l)) / l.max()
    c = dev_checks(Ad, lam, zr, zi, nA=l.max())
    print(f"  eig err={err:.2e} {fmt(c)}", flush=True)
    assert err <= TOL_EIG
    _assert_pairs(c)


def test_c3_bse_10000(h):
    import torch
    m = 5000
    print(f"C3 n={2 * m}", flush=True)
    K, Ab, Bb = wl.bse_shaped(m, 3)
    Lp = np.linalg.cholesky(Ab + Bb)
    ref = np.sqrt(np.sort(np.linalg.eigvalsh(Lp.T @ (Ab - Bb) @ Lp)))
    Kd = to_dev(K)
    del K
    lam, zr, zi = h.solve(Kd)
    torch.cuda.synchronize()
    err = np.max(np.abs(lam.cpu().numpy() - ref)) / ref.max()
    c = dev_checks(Kd, lam, zr, zi, nA=ref.max())
    print(f"  eig err={err:.2e} {fmt(c)}", flush=True)
    assert err <= TOL_EIG
    _assert_pairs(c)


def test_c5_batch_512(h):
    import torch
    sizes, mats = wl.batch(512, 5)
    print(f"C5 batch of {len(sizes)}, n in [{min(sizes)}, {max(sizes)}]", flush=True)
    dev = [to_dev(A) for A in mats]
    res_list, status, st = h.solve_batched(dev)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in status)
    worst = {}
    for Ad, (lam, zr, zi) in zip(dev, res_list):
        c = dev_checks(Ad, lam, zr, zi)
        _assert_pairs(c)
        for k, v in c.items():
            worst[k] = max(worst.get(k, 0.0), v)
    print(f"  worst {fmt(worst)}", flush=True)
    for i in range(0, 512, 64):                    # oracle sample
        lref, _ = oracle.skew_evd(mats[i])
        lam = res_list[i][0].cpu().numpy()
        assert np.max(np.abs(lam - lref)) <= TOL_EIG * lref.max()
