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
