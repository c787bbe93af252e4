"""Full-size GPU checks at the workload sizes (in the same launch configuration
the benchmark times): properties that hold at any size, and exact pins where
the input has a known spectrum.

* C4 n = 16384 random (both forms): global residual and orthogonality (FP64
  products on the GPU with torch, independent of the library), the trace
  identities sum lambda^2 = ||A||_F^2 / 2 and sum lambda^4 = ||A^2||_F^2 / 2
  (they fail if an eigenvalue is missing, duplicated or wrong).
* C2 n = 8192 prescribed spectrum: eigenvalues against the exact l_k.
* C3 n = 10000 BSE-shaped: eigenvalues against sqrt(eig(L+^T (A-B) L+)).
* C5 batch of 512 uneven matrices: residual/orthogonality of every matrix,
  eigenvalues of a sample against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


def _checks(Ad, lam, zr, zi):
    """(residual, orthogonality) with FP64 torch products on the GPU."""
    import torch
    n = Ad.shape[0]
    Af = torch.tril(Ad.contiguous(), -1)
    Af = Af - Af.t()
    zr = zr.contiguous()
    zi = zi.contiguous()
    Rr = Af @ zr + zi * lam[None, :]
    Ri = Af @ zi - zr * lam[None, :]
    nA = lam.max().item()
    res = (Rr.pow(2).sum() + Ri.pow(2).sum()).sqrt().item() / (n * nA)
    del Rr, Ri
    G1 = zr.t() @ zr + zi.t() @ zi
    G1.diagonal().sub_(1.0)
    G2 = zr.t() @ zi - zi.t() @ zr
    orth = (G1.pow(2).sum() + G2.pow(2).sum()).sqrt().item() / n
    del G1, G2
    # trace identities (A normal with eigenvalues +-i lam)
    fro2 = Af.pow(2).sum().item()
    s2 = 2.0 * lam.pow(2).sum().item()
    A2 = Af @ Af
    f4 = A2.pow(2).sum().item()
    s4 = 2.0 * lam.pow(4).sum().item()
    del Af, A2
    torch.cuda.empty_cache()
    return res, orth, abs(s2 / fro2 - 1.0), abs(s4 / f4 - 1.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c4_random_16384(h, precision):
    import torch
    n = 16384
    print(f"C4 n={n} {precision}", flush=True)
    Ad = to_dev(wl.random_skew(n, 4))
    lam, zr, zi = h.solve(Ad, precision=precision)
    torch.cuda.synchronize()
    assert lam.numel() == n // 2
    assert bool((lam[1:] >= lam[:-1]).all()) and lam[0].item() >= 0.0
    res, orth, e2, e4 = _checks(Ad, lam, zr, zi)
    print(f"  res={res:.2e} orth={orth:.2e} trace2={e2:.1e} trace4={e4:.1e} "
          f"sweeps={h.last_info.refine_sweeps}", flush=True)
    assert res <= TOL_RES and orth <= TOL_ORTH
    assert e2 <= 1e-13 and e4 <= 1e-12


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
    res, orth, e2, _ = _checks(Ad, lam, zr, zi)
    print(f"  eig err={err:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
    assert err <= TOL_EIG and res <= TOL_RES and orth <= TOL_ORTH


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
    res, orth, _, _ = _checks(Kd, lam, zr, zi)
    print(f"  eig err={err:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
    assert err <= TOL_EIG and res <= TOL_RES and orth <= TOL_ORTH


def test_c5_batch_512(h):
    import torch
    sizes, mats = wl.batch(512, 5)
    print(f"C5 batch of {len(sizes)}, n in [{min(sizes)}, {max(sizes)}]", flush=True)
    dev = [to_dev(A) for A in mats]
    res_list, status, st = h.solve_batched(dev)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in status)
    worst_r, worst_o = 0.0, 0.0
    for Ad, (lam, zr, zi) in zip(dev, res_list):
        n = Ad.shape[0]
        Af = torch.tril(Ad.contiguous(), -1)
        Af = Af - Af.t()
        Z = torch.complex(zr.contiguous(), zi.contiguous())
        R = torch.complex(Af, torch.zeros_like(Af)) @ Z - Z * (1j * lam)[None, :]
        nA = lam.max().item()
        worst_r = max(worst_r, torch.linalg.norm(R).item() / (n * nA))
        G = Z.conj().t() @ Z
        G.diagonal().sub_(1.0)
        worst_o = max(worst_o, torch.linalg.norm(G).item() / n)
    print(f"  worst res={worst_r:.2e} worst orth={worst_o:.2e}", flush=True)
    assert worst_r <= TOL_RES and worst_o <= TOL_ORTH
    for i in range(0, 512, 64):                    # oracle sample
        lref, _ = oracle.skew_evd(mats[i])
        lam = res_list[i][0].cpu().numpy()
        assert np.max(np.abs(lam - lref)) <= TOL_EIG * lref.max()
