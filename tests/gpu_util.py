"""Helpers for the GPU tests: device inputs, tolerance metrics (FP64, CPU)."""
import numpy as np
import torch

# Tolerances of the parity contract (FP64): eigenvalue error <= 1e-12 ||A||,
# residual ||A Z - Z diag(i lam)||_F / (n ||A||) <= 1e-13,
# orthogonality ||Z^H Z - I||_F / n <= 1e-13.
TOL_EIG = 1e-12
TOL_RES = 1e-13
TOL_ORTH = 1e-13


def to_dev(A):
    """numpy (column-major) -> CUDA float64 tensor holding A column-major."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).cuda()
    return t.t()          # (n, n) view with strides (1, n)


def metrics(A, lam, Z, norm=None):
    """(residual, orthogonality, ||A||) in FP64 on the CPU."""
    n = A.shape[0]
    if norm is None:
        norm = float(np.max(lam)) if lam.size else 0.0
    norm = max(norm, 1e-300)
    R = A @ Z - Z * (1j * lam)[None, :]
    res = np.linalg.norm(R) / (n * norm)
    orth = np.linalg.norm(Z.conj().T @ Z - np.eye(Z.shape[1])) / n
    return res, orth, norm


def solve_np(h, A, nev=None, **kw):
    lam, zr, zi = h.solve(to_dev(A), nev=nev, **kw)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), zr.cpu().numpy() + 1j * zi.cpu().numpy()


def band_to_dense(band, n, b):
    B = np.zeros((n, n))
    for j in range(n):
        for d in range(1, b + 1):
            if j + d < n:
                B[j + d, j] = band[d, j]
                B[j, j + d] = -band[d, j]
    return B


def phase_match(Z, Zref, lam, gap_tol, tol):
    """For eigenvalues separated by more than gap_tol from their neighbours,
    |<z_ref, z>| >= 1 - tol (eigenvectors agree up to a unit phase)."""
    worst = 0.0
    for k in range(len(lam)):
        lo = lam[k - 1] if k > 0 else -np.inf
        hi = lam[k + 1] if k + 1 < len(lam) else np.inf
        gap = min(lam[k] - lo, hi - lam[k], 2 * lam[k] if lam[k] > 0 else np.inf)
        if gap > gap_tol:
            worst = max(worst, 1.0 - abs(np.vdot(Zref[:, k], Z[:, k])))
    return worst <= tol, worst


def dev_checks(Ad, lam, zr, zi, nA=None):
    """Accuracy measures with FP64 torch products on the GPU (independent of
    the library), for full-size inputs:
      res    ||A Z - Z diag(i lam)||_F / (n ||A||)
      colres max_k ||A z_k - i lam_k z_k||_2 / ||A||  (for normal A each lam_k
             then lies within colres * ||A|| of an eigenvalue)
      orth   ||Z^H Z - I||_F / n,  orth_max  max |Z^H Z - I|
      tr2, tr4  relative errors of sum lam^2 = ||A||_F^2 / 2 and
             sum lam^4 = ||A^2||_F^2 / 2
    ||A|| = nA, default max lam."""
    n = Ad.shape[0]
    Af = torch.tril(Ad.contiguous(), -1)
    Af = Af - Af.t()
    zr = zr.contiguous()
    zi = zi.contiguous()
    nA = lam.max().item() if nA is None else nA
    Rr = Af @ zr + zi * lam[None, :]
    Ri = Af @ zi - zr * lam[None, :]
    col2 = Rr.pow(2).sum(0) + Ri.pow(2).sum(0)
    res = col2.sum().sqrt().item() / (n * nA)
    colres = col2.max().sqrt().item() / nA
    del Rr, Ri, col2
    G1 = zr.t() @ zr + zi.t() @ zi
    G1.diagonal().sub_(1.0)
    G2 = zr.t() @ zi - zi.t() @ zr
    orth = (G1.pow(2).sum() + G2.pow(2).sum()).sqrt().item() / n
    orth_max = max(G1.abs().max().item(), G2.abs().max().item())
    del G1, G2
    fro2 = Af.pow(2).sum().item()
    s2 = 2.0 * lam.pow(2).sum().item()
    A2 = Af @ Af
    f4 = A2.pow(2).sum().item()
    s4 = 2.0 * lam.pow(4).sum().item()
    del Af, A2
    torch.cuda.empty_cache()
    tr2 = abs(s2 / fro2 - 1.0) if fro2 > 0 else abs(s2)
    tr4 = abs(s4 / f4 - 1.0) if f4 > 0 else abs(s4)
    return {"res": res, "colres": colres, "orth": orth, "orth_max": orth_max, "tr2": tr2, "tr4": tr4}


def fmt(d):
    return " ".join(f"{k}={v:.2e}" for k, v in d.items())
