"""GPU test of the allocation-free entry point skew_evd_noalloc (through the
C-ABI): its results are bitwise equal to those of skew_evd_ex with default
options on the same inputs, on two calls in a row (the second with a smaller
order, so the shared scratch array holds the previous call's contents), and
orders above its limit are refused with NOMEM before any device work."""
import ctypes

import numpy as np
import pytest

from paper_1912_04062_amd import workloads as wl

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lib, Ad, nev, stream):
    import torch
    from paper_1912_04062_amd import skewevd
    n = Ad.shape[0]
    Ac, lda = skewevd.colmajor(Ad)
    lam = torch.full((max(nev, 1),), float("nan"), dtype=torch.float64, device="cuda")
    zr = skewevd.empty_colmajor(n, max(nev, 1), "cuda").fill_(float("nan"))
    zi = skewevd.empty_colmajor(n, max(nev, 1), "cuda").fill_(float("nan"))
    st = lib.skew_evd_noalloc(n, ctypes.c_void_p(Ac.data_ptr()), lda, nev, ctypes.c_void_p(lam.data_ptr()),
                              ctypes.c_void_p(zr.data_ptr()), zr.stride(1), ctypes.c_void_p(zi.data_ptr()),
                              zi.stride(1), ctypes.c_void_p(stream.cuda_stream))
    return st, lam[:nev], zr[:, :nev], zi[:, :nev]


def test_noalloc_matches_skew_evd_ex():
    import torch
    from paper_1912_04062_amd import skewevd
    lib = skewevd.lib()
    h = skewevd.Handle()
    stream = torch.cuda.current_stream()
    nmax = lib.skew_evd_noalloc_max_n()
    assert nmax >= 512
    for n, seed in ((nmax, 11), (301, 12)):          # the second call is smaller
        print(f"noalloc n={n}", flush=True)
        Ad = to_dev(wl.random_skew(n, seed))
        nev = (n + 1) // 2
        st, lam, zr, zi = _noalloc(lib, Ad, nev, stream)
        torch.cuda.synchronize()
        assert st == 0, skewevd.status_string(st)
        l1, r1, i1 = h.solve(Ad)
        torch.cuda.synchronize()
        assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1)
    # above the limit: refused, outputs untouched
    Ad = to_dev(wl.random_skew(nmax + 1, 13))
    st, lam, _, _ = _noalloc(lib, Ad, (nmax + 2) // 2, stream)
    torch.cuda.synchronize()
    assert st == skewevd.ERR_NOMEM
    assert "allocation-free" in skewevd.status_string(st)
    assert bool(torch.isnan(lam).all())
    h.close()
