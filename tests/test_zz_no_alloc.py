"""GPU test of the allocation-free entry point skew_evd_noalloc (through the
C-ABI): its results are bitwise equal to those of skew_evd_ex with default
options on the same inputs, on two calls in a row (the second with a smaller
order, so the shared scratch array holds the previous call's contents), and
an order above its limit is refused with NOMEM before any device work."""
import pytest

from paper_1912_04062_amd import workloads as wl

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _filled(n, nev):
    import torch
    from paper_1912_04062_amd import skewevd
    return (torch.full((max(nev, 1),), float("nan"), dtype=torch.float64, device="cuda"),
            skewevd.empty_colmajor(n, max(nev, 1), "cuda").fill_(float("nan")),
            skewevd.empty_colmajor(n, max(nev, 1), "cuda").fill_(float("nan")))


def test_noalloc_matches_skew_evd_ex():
    import torch
    from paper_1912_04062_amd import skewevd
    h = skewevd.Handle()
    nmax = skewevd.noalloc_max_n()
    assert nmax >= 512
    for n, seed in ((nmax, 11), (301, 12)):          # the second call is smaller
        print(f"noalloc n={n}", flush=True)
        Ad = to_dev(wl.random_skew(n, seed))
        nev = (n + 1) // 2
        st, lam, zr, zi = skewevd.solve_noalloc(Ad, nev, out=_filled(n, nev))
        torch.cuda.synchronize()
        assert st == 0, skewevd.status_string(st)
        l1, r1, i1 = h.solve(Ad)
        torch.cuda.synchronize()
        assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1)
    # a partial spectrum on a side stream
    s2 = torch.cuda.Stream()
    Ad = to_dev(wl.random_skew(200, 14))
    with torch.cuda.stream(s2):
        st, lam, zr, zi = skewevd.solve_noalloc(Ad, 30, out=_filled(200, 30), stream=s2)
    s2.synchronize()
    assert st == 0
    l1, r1, i1 = h.solve(Ad, nev=30)
    torch.cuda.synchronize()
    assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1)
    # above the limit: refused, outputs untouched
    n = nmax + 1
    Ad = to_dev(wl.random_skew(n, 13))
    out = _filled(n, (n + 1) // 2)
    st, lam, _, _ = skewevd.solve_noalloc(Ad, out=out)
    torch.cuda.synchronize()
    assert st == skewevd.ERR_NOMEM
    assert "allocation-free" in skewevd.status_string(st)
    assert bool(torch.isnan(lam).all())
    h.close()
