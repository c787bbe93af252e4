"""GPU edge cases of the solver through the C-ABI.

* Clusters wider than the fixed Gram-Schmidt window (1024 vectors) at
  nev > 2048: the zero matrix, a prescribed spectrum with two eigenvalues of
  multiplicity 2048 each, and a tridiagonal input that splits into identical
  blocks.  Every eigenvalue is known exactly; orthogonality is asserted both
  normalized (||Z^H Z - I||_F / n <= 1e-13) and entrywise (<= 1e-12).
* Padded leading dimensions (lda > n, ldz > n) on input and outputs.
* Workspace contents: a solve on a workspace filled with NaN bytes and one on
  a zeroed workspace give bitwise equal results (no kernel reads workspace it
  has not written), in both forms and with the second stream in use.
* Error paths forced from the host: the inverse iteration's convergence test
  (debug hook) reports NOCONV; the batched form refuses the precision form.
"""
import numpy as np
import pytest

from paper_1912_04062_amd import workloads as wl

from gpu_util import TOL_EIG, TOL_ORTH, TOL_RES, dev_checks, fmt, metrics, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_1912_04062_amd import skewevd
    return skewevd.Handle()


def _wide(h, A, exact, label):
    import torch
    n = A.shape[0]
    Ad = to_dev(A)
    lam, zr, zi = h.solve(Ad)
    torch.cuda.synchronize()
    nA = max(float(np.max(exact)), 1.0)
    err = np.max(np.abs(lam.cpu().numpy() - exact)) / nA
    c = dev_checks(Ad, lam, zr, zi, nA=nA)
    print(f"  {label}: eig err={err:.2e} {fmt(c)}", flush=True)
    assert err <= TOL_EIG
    assert c["res"] <= TOL_RES and c["colres"] <= 1e-12
    assert c["orth"] <= TOL_ORTH and c["orth_max"] <= 1e-12
    return lam


def test_cluster_zero_matrix_8192(h):
    n = 8192
    print(f"zero matrix n={n}", flush=True)
    lam = _wide(h, np.zeros((n, n), order="F"), np.zeros(n // 2), "zero")
    assert bool((lam == 0).all())


def test_cluster_repeated_eigenvalues_8192(h):
    n = 8192
    print(f"repeated l_k n={n}", flush=True)
    l = np.repeat([1.0, 2.0], n // 4)           # two clusters of 2048 vectors
    A, l = wl.prescribed_large(n, 61, l=l)
    _wide(h, A, l, "repeated")


def test_cluster_identical_tridiagonal_blocks_8192(h):
    n = 8192
    print(f"identical tridiagonal blocks n={n}", flush=True)
    pat = [1.0, 2.0, 3.0]                        # blocks of order 4
    A = wl.tridiag_blocks(n, pat)
    T = np.diag(pat, 1) + np.diag(pat, -1)
    ev = np.sort(np.linalg.eigvalsh(T))[2:]      # the two non-negative ones
    exact = np.repeat(ev, n // 4)                # each 2048 times
    _wide(h, A, exact, "blocks")


@pytest.mark.parametrize("n", [333, 1200])
def test_padded_leading_dimensions(h, n):
    import torch
    from paper_1912_04062_amd import skewevd
    print(f"padded lda/ldz n={n}", flush=True)
    A = wl.random_skew(n, 70 + n)
    big = np.full((n + 5, n + 3), np.nan, order="F")   # padding never read
    big[:n, :n] = A
    Abig = to_dev(big)                                 # lda = n + 5
    Av = Abig[:n, :n]
    nev = (n + 1) // 2
    lam = torch.empty(nev, dtype=torch.float64, device="cuda")
    zr = skewevd.empty_colmajor(n + 7, nev, "cuda")
    zi = skewevd.empty_colmajor(n + 11, nev, "cuda")
    zr.fill_(7.0)
    zi.fill_(-7.0)
    l1, r1, i1 = h.solve(Av, out=(lam, zr[:n], zi[:n]))
    torch.cuda.synchronize()
    assert r1.stride(1) == n + 7 and i1.stride(1) == n + 11
    l0, r0, i0 = h.solve(to_dev(A))
    torch.cuda.synchronize()
    assert torch.equal(l1, l0) and torch.equal(r1, r0) and torch.equal(i1, i0)
    assert bool((zr[n:] == 7.0).all()) and bool((zi[n:] == -7.0).all())   # rows past n untouched
    lam_np = l1.cpu().numpy()
    Z = r1.cpu().numpy() + 1j * i1.cpu().numpy()
    res, orth, _ = metrics(A, lam_np, Z)
    assert res <= TOL_RES and orth <= TOL_ORTH


@pytest.mark.parametrize("n,precision", [(1500, "fp64"), (4100, "fp64"), (1500, "fp32"), (4100, "fp32")])
def test_workspace_contents_do_not_matter(h, n, precision):
    """NaN-filled versus zeroed workspace: bitwise equal outputs.  n = 4100
    uses the second stream (T factors beside the inverse iteration)."""
    import torch
    from paper_1912_04062_amd import skewevd
    print(f"workspace NaN vs zero n={n} {precision}", flush=True)
    Ad = to_dev(wl.random_skew(n, 80 + n))
    outs = []
    for dbg in (skewevd.DEBUG_NAN_WS, skewevd.DEBUG_ZERO_WS, skewevd.DEBUG_NAN_WS):
        o = skewevd.default_opts(precision, debug=dbg)
        lam, zr, zi = h.solve(Ad, opts=o)
        torch.cuda.synchronize()
        outs.append((lam.clone(), zr.clone(), zi.clone(), h.last_info.refine_sweeps))
    print(f"  sweeps {[x[3] for x in outs]}", flush=True)
    for k in (1, 2):
        assert outs[k][3] == outs[0][3]
        for a, b in zip(outs[0][:3], outs[k][:3]):
            assert torch.equal(a, b)
    assert bool(torch.isfinite(outs[0][1]).all())


def test_invit_noconv_reported(h):
    from paper_1912_04062_amd import skewevd
    A = wl.random_skew(200, 91)
    o = skewevd.default_opts(debug=skewevd.DEBUG_INVIT_NOCONV)
    with pytest.raises(skewevd.SkewEvdError) as e:
        h.solve(to_dev(A), opts=o)
    assert e.value.status == skewevd.ERR_NOCONV
    assert "inverse iteration" in skewevd.status_string(skewevd.ERR_NOCONV)
    lam, _, _ = h.solve(to_dev(A))                  # the handle still works
    assert np.isfinite(lam.cpu().numpy()).all()


def test_batched_refuses_precision_form(h):
    mats = [to_dev(wl.random_skew(100, 1))]
    _, _, st = h.solve_batched(mats, precision="fp32")
    assert st == -10


@pytest.mark.skip(reason="two benchmark runs of the batched precision form ended in a host "
                         "segmentation fault at process exit whose cause is not shown; the "
                         "batched form refuses the precision form (argument -10) until it is")
def test_batched_precision_form():
    pass


def test_batched_graph_replays(h):
    """The batched form captures its launches as a HIP graph on the first call
    of a batch signature and replays it on later calls with the same inputs
    and outputs.  Three calls in a row, with the program's own eager work
    (single solves of the same problems) and synchronizations between them:
    every replay bitwise equal to the single solves.  A call with other
    output buffers captures a new graph, with the same results."""
    import torch
    from paper_1912_04062_amd import skewevd
    print("batched graph replays", flush=True)
    sizes = [5, 64, 65, 130, 200, 257, 300, 511, 64, 900]
    mats = [wl.random_skew(n, 610 + k) for k, n in enumerate(sizes)]
    dev = [to_dev(A) for A in mats]
    ref = []
    for Ad in dev:
        l1, r1, i1 = h.solve(Ad)
        ref.append((l1.clone(), r1.clone(), i1.clone()))
    torch.cuda.synchronize()
    out = h.batched_outputs(dev)
    for rep in range(3):
        for o in out:                     # stale contents must not matter
            for t in o:
                t.fill_(float("nan"))
        res, status, st = h.solve_batched(dev, out=out)
        torch.cuda.synchronize()
        assert st == 0 and all(x == 0 for x in status), (rep, status)
        for k, ((lam, zr, zi), (l1, r1, i1)) in enumerate(zip(res, ref)):
            assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1), (rep, k)
        # eager work between the replays
        l2, _, _ = h.solve(dev[3])
        torch.cuda.synchronize()
        assert torch.equal(l2, ref[3][0])
    res, status, st = h.solve_batched(dev)          # fresh outputs: a new capture
    torch.cuda.synchronize()
    assert st == 0
    for k, ((lam, zr, zi), (l1, r1, i1)) in enumerate(zip(res, ref)):
        assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1), k


def test_batched_mixed_problems(h):
    """One batched call over problems of every kind: tiny orders, a partial
    spectrum, an order above the batched path's limit (solved on its own), a
    degenerate cluster (flagged on the device and solved again on its own), a
    zero matrix and a non-finite input (its own status, the others unaffected).
    Every result is bitwise equal to the single solve of the same problem."""
    import torch
    from paper_1912_04062_amd import skewevd
    print("batched mixed", flush=True)
    mats, nevs = [], []
    for n in (1, 2, 3, 65, 300):
        mats.append(wl.random_skew(n, 500 + n))
        nevs.append((n + 1) // 2)
    mats.append(wl.random_skew(301, 77))
    nevs.append(40)                                   # partial spectrum
    mats.append(wl.tridiag_blocks(1024, [1.0, 2.0, 3.0]))
    nevs.append(512)                                  # two clusters of 256
    mats.append(np.zeros((200, 200), order="F"))
    nevs.append(100)
    bad = wl.random_skew(128, 3)
    bad[70, 5] = np.inf
    mats.append(bad)
    nevs.append(64)
    mats.append(wl.random_skew(4100, 8))              # above the batched path's limit
    nevs.append(2050)
    dev = [to_dev(A) for A in mats]
    res, status, st = h.solve_batched(dev, nevs=nevs)
    torch.cuda.synchronize()
    print(f"  status {status} -> {st}", flush=True)
    assert st == skewevd.ERR_NONFINITE
    for k, (A, Ad, nv, (lam, zr, zi), s) in enumerate(zip(mats, dev, nevs, res, status)):
        if k == 8:
            assert s == skewevd.ERR_NONFINITE
            continue
        assert s == 0, (k, s)
        l1, r1, i1 = h.solve(Ad, nev=nv)
        torch.cuda.synchronize()
        assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1), k
        if A.shape[0] > 1:
            c = dev_checks(Ad, lam, zr, zi, nA=max(lam.max().item(), 1.0))
            assert c["colres"] <= 1e-12 and c["orth_max"] <= 1e-12, (k, c)


def test_batched_empty_spectra(h):
    """Problems asking for no eigenpairs beside ones that do: the batched
    tridiagonal launches map workgroups to problems through prefix tables of
    their block counts, in which a problem without eigenpairs has none.  The
    others are bitwise equal to their single solves."""
    import torch
    print("batched empty spectra", flush=True)
    sizes = [64, 65, 300, 2, 257, 130]
    nevs = [0, 33, 0, 1, 0, 40]
    mats = [wl.random_skew(n, 640 + k) for k, n in enumerate(sizes)]
    dev = [to_dev(A) for A in mats]
    res, status, st = h.solve_batched(dev, nevs=nevs)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in status), status
    for k, (Ad, nv, (lam, zr, zi)) in enumerate(zip(dev, nevs, res)):
        assert lam.numel() == nv and zr.shape[1] == nv, k
        if nv == 0:
            continue
        l1, r1, i1 = h.solve(Ad, nev=nv)
        torch.cuda.synchronize()
        assert torch.equal(lam, l1) and torch.equal(zr, r1) and torch.equal(zi, i1), k


@pytest.mark.parametrize("n,precision", [(300, "fp64"), (301, "fp64"), (257, "fp32")])
def test_all_pairs(h, n, precision):
    """opts.all_pairs: every eigenpair of both signs, ascending, the exact zero
    of odd n once; the n vectors are orthonormal (conj(z) of +lambda is the
    vector of -lambda, orthogonal to z) and match the oracle's spectrum."""
    import oracle
    import torch
    from paper_1912_04062_amd import skewevd
    print(f"all pairs n={n} {precision}", flush=True)
    A = wl.random_skew(n, 600 + n)
    o = skewevd.default_opts(precision, all_pairs=1)
    mu, zr, zi = h.solve(to_dev(A), opts=o)
    torch.cuda.synchronize()
    mu = mu.cpu().numpy()
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    assert mu.shape == (n,) and Z.shape == (n, n)
    lref, _ = oracle.skew_evd(A)
    full = np.concatenate([-lref[::-1][: n - len(lref)], lref])
    nA = lref.max()
    assert np.all(np.diff(mu) >= 0)
    assert np.max(np.abs(mu - full)) <= TOL_EIG * nA
    if n % 2:
        assert mu[n // 2] == 0.0
    assert np.array_equal(mu[: n // 2], -mu[::-1][: n // 2])
    res, orth, _ = metrics(A, mu, Z, nA)
    print(f"  res={res:.2e} orth={orth:.2e}", flush=True)
    assert res <= TOL_RES and orth <= TOL_ORTH


@pytest.mark.parametrize("n,pm", [(300, 1), (300, 2), (1100, 1), (1100, 2), (2049, 2)])
def test_panel_methods(h, n, pm):
    """Both panel factorizations of the full-to-band stage (Cholesky QR twice
    with reconstruction, and the column-by-column Householder kernel) give
    eigenpairs within the FP64 tolerances of the oracle."""
    import oracle
    import torch
    from paper_1912_04062_amd import skewevd
    print(f"panel method {pm} n={n}", flush=True)
    A = wl.random_skew(n, 900 + n)
    lam, zr, zi = h.solve(to_dev(A), opts=skewevd.default_opts(panel_method=pm))
    torch.cuda.synchronize()
    lam = lam.cpu().numpy()
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    lref, _ = oracle.skew_evd(A)
    nA = lref.max()
    assert np.max(np.abs(lam - lref)) <= TOL_EIG * nA
    res, orth, _ = metrics(A, lam, Z, nA)
    assert res <= TOL_RES and orth <= TOL_ORTH


def _route_vs_oracle(h, A, reduction, label):
    import oracle
    import torch
    from paper_1912_04062_amd import skewevd
    n = A.shape[0]
    lam, zr, zi = h.solve(to_dev(A), opts=skewevd.default_opts(reduction=reduction))
    torch.cuda.synchronize()
    lam = lam.cpu().numpy()
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    lref, _ = oracle.skew_evd(A)
    nA = max(lref.max(), 1.0) if n > 1 else 1.0
    err = np.max(np.abs(lam - lref)) / nA
    if n > 1:
        res, orth, _ = metrics(A, lam, Z, nA)
        print(f"  {label}: eig err={err:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
        assert res <= TOL_RES and orth <= TOL_ORTH
    assert err <= TOL_EIG


@pytest.mark.parametrize("n", [1, 2, 3, 65, 130, 300, 1001, 2050, 4100])
def test_one_stage_route(h, n):
    """The one-stage reduction (Section 2.3.1) with its one-stage
    back-transformation: eigenpairs within the FP64 tolerances of the oracle,
    ragged last panels and n above the fixed Gram-Schmidt window included."""
    print(f"one-stage n={n}", flush=True)
    _route_vs_oracle(h, wl.random_skew(n, 1700 + n), 1, "one-stage")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 65, 130, 300, 1001, 2050])
def test_complex_hermitian_route(h, n):
    """The complex Hermitian route on iA (the comparison of the introduction
    and Section 4.1): complex one-stage reduction, the real tridiagonal
    matrix with its diagonal, complex back-transformation; eigenpairs within
    the FP64 tolerances of the oracle in the skew solver's form."""
    print(f"complex Hermitian n={n}", flush=True)
    _route_vs_oracle(h, wl.random_skew(n, 1900 + n), 2, "complex")


@pytest.mark.parametrize("reduction", [1, 2])
def test_one_stage_routes_partial_padded_all_pairs(h, reduction):
    """Both one-stage routes with a partial spectrum, with padded leading
    dimensions (bitwise equal to the unpadded solve, padding never read or
    written), and with every eigenpair (both signs)."""
    import oracle
    import torch
    from paper_1912_04062_amd import skewevd
    n = 301
    print(f"routes: partial/padded/all pairs, reduction {reduction}", flush=True)
    A = wl.random_skew(n, 2300 + reduction)
    lref, _ = oracle.skew_evd(A)
    nA = lref.max()
    o = skewevd.default_opts(reduction=reduction)
    # partial spectrum: the nev smallest non-negative eigenvalues
    lam, zr, zi = h.solve(to_dev(A), nev=40, opts=o)
    torch.cuda.synchronize()
    assert np.max(np.abs(lam.cpu().numpy() - lref[:40])) <= TOL_EIG * nA
    c = dev_checks(to_dev(A), lam, zr, zi, nA=nA)
    assert c["colres"] <= 1e-12 and c["orth_max"] <= 1e-12, c
    # padded leading dimensions
    big = np.full((n + 5, n + 3), np.nan, order="F")
    big[:n, :n] = A
    Av = to_dev(big)[:n, :n]
    nev = (n + 1) // 2
    lamp = torch.empty(nev, dtype=torch.float64, device="cuda")
    zrp = skewevd.empty_colmajor(n + 7, nev, "cuda")
    zip_ = skewevd.empty_colmajor(n + 11, nev, "cuda")
    zrp.fill_(7.0)
    zip_.fill_(-7.0)
    l1, r1, i1 = h.solve(Av, out=(lamp, zrp[:n], zip_[:n]), opts=o)
    l0, r0, i0 = h.solve(to_dev(A), opts=o)
    torch.cuda.synchronize()
    assert torch.equal(l1, l0) and torch.equal(r1, r0) and torch.equal(i1, i0)
    assert bool((zrp[n:] == 7.0).all()) and bool((zip_[n:] == -7.0).all())
    # every eigenpair: signed values ascending, conj vectors for the negative half
    oa = skewevd.default_opts(reduction=reduction, all_pairs=1)
    la, ra, ia = h.solve(to_dev(A), opts=oa)
    torch.cuda.synchronize()
    mu = la.cpu().numpy()
    ref = np.concatenate([-lref[::-1][: n - len(lref)], lref])
    assert np.all(np.diff(mu) >= 0)
    assert np.max(np.abs(mu - ref)) <= TOL_EIG * nA
    Z = ra.cpu().numpy() + 1j * ia.cpu().numpy()
    Af = np.tril(A, -1) - np.tril(A, -1).T
    R = Af @ Z - Z * (1j * mu)[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-12 * nA
    G = Z.conj().T @ Z - np.eye(n)
    assert np.max(np.abs(G)) <= 1e-12


def test_complex_hermitian_route_prescribed(h):
    """Known spectrum with close pairs (prescribed l_k) through the complex
    route: every eigenvalue against l_k."""
    import torch
    from paper_1912_04062_amd import skewevd
    n = 700
    A, l, _ = wl.prescribed(n, 23)
    lam, zr, zi = h.solve(to_dev(A), opts=skewevd.default_opts(reduction=2))
    torch.cuda.synchronize()
    exact = np.sort(l)
    nA = exact.max()
    err = np.max(np.abs(np.sort(lam.cpu().numpy()) - exact)) / nA
    Z = zr.cpu().numpy() + 1j * zi.cpu().numpy()
    res, orth, _ = metrics(A, lam.cpu().numpy(), Z, nA)
    print(f"  prescribed n={n}: eig err={err:.2e} res={res:.2e} orth={orth:.2e}", flush=True)
    assert err <= TOL_EIG and res <= TOL_RES and orth <= TOL_ORTH


@pytest.mark.parametrize("reduction", [1, 2])
def test_one_stage_routes_workspace_contents(h, reduction):
    """NaN-filled versus zeroed workspace, bitwise equal, for both one-stage
    routes (a ragged last panel included)."""
    import torch
    from paper_1912_04062_amd import skewevd
    print(f"workspace NaN vs zero, reduction {reduction}", flush=True)
    Ad = to_dev(wl.random_skew(333, 97))
    outs = []
    for dbg in (skewevd.DEBUG_NAN_WS, skewevd.DEBUG_ZERO_WS):
        lam, zr, zi = h.solve(Ad, opts=skewevd.default_opts(reduction=reduction, debug=dbg))
        torch.cuda.synchronize()
        outs.append((lam.clone(), zr.clone(), zi.clone()))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    assert bool(torch.isfinite(outs[0][1]).all())


def test_unbuilt_options_are_argument_errors(h):
    """The boundary's BF16 precision value and tridiagonal-method values other
    than bisection + inverse iteration are refused as argument errors."""
    from paper_1912_04062_amd import skewevd
    A = to_dev(wl.random_skew(100, 6))
    h.solve(A, opts=skewevd.default_opts(precision=2), check=False)
    assert h.last_status == -11
    o = skewevd.default_opts()
    o.tridiag_method = 1
    h.solve(A, opts=o, check=False)
    assert h.last_status == -11
    lam, _, _ = h.solve(A)                   # the handle still works
    assert np.isfinite(lam.cpu().numpy()).all()


@pytest.mark.parametrize("reduction", [1, 2])
def test_one_stage_argument_rules(h, reduction):
    from paper_1912_04062_amd import skewevd
    A = to_dev(wl.random_skew(100, 5))
    for kw in ({"precision": "fp32"}, {"band": 32}):
        h.solve(A, opts=skewevd.default_opts(reduction=reduction, **kw), check=False)
        assert h.last_status == -11, kw
    _, _, st = h.solve_batched([A], reduction=reduction)
    assert st == -10
