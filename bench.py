"""Benchmark: skew-symmetric eigensolver time-to-solution on one MI355X.

One step = one complete solve (every stage: full-to-band, bulge chase,
tridiagonal solve, D scaling, both back-transformations, and for the precision
form the refinement) of a dense random skew-symmetric A of order n = 16384
(A = (B - B^T)/2, B iid N(0, 1), seed 4) with n/2 eigenpairs, inputs resident
in HBM.  value = useful FLOP rate F / time, F = (4/3) n^3 + 8 n^2 nev (the
tridiagonalization plus two back-transformations of 2*nev real columns).

Prints ONE JSON line (rank 0).  The roofline object describes the kernel that
takes the largest share of the step, timed with HIP events on the library's
stream; cpu_baseline is the FP64 oracle timed on a bounded sample on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3}          # TFLOP/s, dense MFMA/vector
HBM_PEAK = 8000.0                           # GB/s


def traffic_record(stage):
    """HBM bytes per launch of the kernel behind `stage`, from a committed
    counter profile (profiles/traffic_*.md: FETCH_SIZE and WRITE_SIZE passes
    scaled by a plain copy of known size), or None when there is none or when
    the kernel's source region has changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record: "):
                    continue
                rec = json.loads(line[len("traffic-record: "):])
                if rec.get("stage") != stage:
                    continue
                with open(os.path.join(ROOT, rec["source"])) as g:
                    src = g.read()
                i, j = src.find(rec["region_begin"]), src.find(rec["region_end"])
                if i < 0 or j < i:
                    return None
                if hashlib.sha256(src[i:j].encode()).hexdigest() != rec["region_sha256"]:
                    return None
                return rec["traffic_bytes"]
    return None


def useful_flops(n, nev):
    return 4.0 / 3.0 * n ** 3 + 8.0 * n * n * nev


def host_cpu():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(sample_n=3072):
    import oracle
    from paper_1912_04062_amd import workloads
    A = workloads.random_skew(sample_n, 4)
    t0 = time.perf_counter()
    oracle.skew_evd(A)
    dt = time.perf_counter() - t0
    f = useful_flops(sample_n, (sample_n + 1) // 2)
    return {"value": f / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one full oracle solve of a random skew matrix n={sample_n} "
                      f"(nev={(sample_n + 1) // 2}), {dt:.1f} s on {host_cpu()}; TFLOP/s with the same "
                      f"useful-flop count F(n) as the GPU line"}


def accuracy(Ad, lam, zr, zi):
    """Residual ||AZ - Z diag(i lam)||_F/(n ||A||) and orthogonality ||Z^H Z - I||_F/n
    with FP64 torch products (outside the timed region)."""
    import torch
    n = Ad.shape[0]
    Af = torch.tril(Ad.contiguous(), -1)
    Af = Af - Af.t()
    zr = zr.contiguous()
    zi = zi.contiguous()
    Rr = Af @ zr + zi * lam[None, :]
    Ri = Af @ zi - zr * lam[None, :]
    res = (Rr.pow(2).sum() + Ri.pow(2).sum()).sqrt().item() / (n * lam.max().item())
    del Rr, Ri, Af
    G1 = zr.t() @ zr + zi.t() @ zi
    G1.diagonal().sub_(1.0)
    G2 = zr.t() @ zi - zi.t() @ zr
    orth = (G1.pow(2).sum() + G2.pow(2).sum()).sqrt().item() / n
    del G1, G2
    torch.cuda.empty_cache()
    return {"residual": res, "orthogonality": orth}


def batch_bench(args):
    """--workload batch: 512 dense random skew matrices of uneven order n ~ U{64..1024}
    (seed 5), ceil(n/2) eigenpairs each, solved by one skew_evd_batched call per step.
    Timed variants: FP64 and FP32 + refinement, each with the fixed band rule and with
    autotuned band widths (tuning, and the capture of the batch's launch graph that the timed
    calls replay, happen in the untimed warm-up call).  value = sum of
    the useful flops F(n_i) over the batch / wall time of the call."""
    import torch
    from paper_1912_04062_amd import skewevd, workloads

    if args.precision == "fp32":
        # the batched entry point accepts the FP64 form only
        raise SystemExit("--workload batch: only --precision fp64 is available")
    sizes, mats = workloads.batch(512, 5)
    dev = [torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t() for A in mats]
    del mats
    F = sum(useful_flops(x, (x + 1) // 2) for x in sizes)
    results = {}
    tunes = {"0": (0,), "1": (1,), "both": (0, 1)}[args.autotune]
    for form in ["fp64"]:
        for tune in tunes:
            h = skewevd.Handle()
            out = h.batched_outputs(dev)
            try:
                for _ in range(max(args.warmup, 1)):
                    res, status, st = h.solve_batched(dev, precision=form, autotune=tune, out=out)
                torch.cuda.synchronize()
                # status 3 (WARN_REFINE): refinement stopped above its own tolerance;
                # the results are valid and the accuracy check below judges them
                if any(x not in (skewevd.OK, skewevd.WARN_REFINE) for x in status):
                    raise RuntimeError(f"batched solve {form} autotune={tune}: status {st}")
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    res, status, st = h.solve_batched(dev, precision=form, autotune=tune, out=out)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / args.steps
            except BaseException:
                h.close()
                raise
            worst = {"residual": 0.0, "orthogonality": 0.0}
            if args.check:                                   # untimed
                for Ad, r in zip(dev, res):
                    a = accuracy(Ad, *r)
                    for k in worst:
                        worst[k] = max(worst[k], a[k])
            bands = {}
            if tune:
                for c in sorted({(x + 127) // 128 for x in sizes}):
                    bands[f"n<={128 * c}"] = h.autotune(128 * c, form)[0]
            key = f"{form}{'_autotuned' if tune else ''}"
            results[key] = {"ms_per_step": wall * 1e3, "tflops": F / wall / 1e12,
                            "accuracy": worst if args.check else None, "bands": bands or None,
                            "warn_refine": sum(1 for x in status if x == skewevd.WARN_REFINE)}
            h.close()

    def ok(k):
        a = results[k]["accuracy"]
        return a is None or (a["residual"] <= 1e-13 and a["orthogonality"] <= 1e-13)

    best = min((k for k in results if ok(k)), key=lambda k: results[k]["ms_per_step"],
               default=next(iter(results)))
    line = {
        "metric": "skew-EVD batch of 512 uneven matrices, ceil(n/2) eigvecs each, TFLOP/s",
        "value": results[best]["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": results[best]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if best.startswith("fp64") else "f32+f64", "data": "synthetic",
        "config": {"workload": "batch of 512 dense random skew matrices A=(B-B^T)/2, B iid N(0,1), "
                               f"n ~ U{{64..1024}} (seed 5), nev=ceil(n/2); reported variant: {best}",
                   "count": len(sizes), "n_min": min(sizes), "n_max": max(sizes),
                   "sum_n3": float(sum(float(x) ** 3 for x in sizes)), "useful_flops": F},
        "variants": results,
    }
    print(json.dumps(line), flush=True)


def start_study(args):
    """--workload start: how far the FP32 pipeline's eigenpairs are from the FP64
    ones before any refinement, next to the gaps of the spectrum.  The FP32 form
    runs with no refinement sweep and no FP64 fallback (WARN_REFINE, the
    unrefined vectors); r0 is its first measured error (largest |I - X^T X|
    entry or off-diagonal |X^T A X| / lambda_max).  A Newton step of the
    refinement is only valid for pairs whose correction r / (relative gap) stays
    well below 1 (the solver refuses corrections above 0.25); the line reports
    how many adjacent pairs that excludes for r0 and for r0 scaled to BF16's
    unit roundoff (2^-8 against FP32's 2^-24, the same pipeline in BF16)."""
    import torch
    from paper_1912_04062_amd import skewevd, workloads
    n = args.n
    A = workloads.random_skew(n, 4)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    del A
    h = skewevd.Handle()
    o = skewevd.default_opts("fp32", max_refine_sweeps=0, no_fp64_fallback=1)
    lam, zr, zi = h.solve(Ad, opts=o)
    torch.cuda.synchronize()
    r0 = h.last_info.refine_residual
    acc = accuracy(Ad, lam, zr, zi)
    lam64, _, _ = h.solve(Ad)
    torch.cuda.synchronize()
    l = lam64.cpu().numpy()
    lmax = float(l.max())
    gap = np.diff(np.concatenate([[-l[0]], l]))   # the pair's distance to its neighbour (and to -lambda_0)
    rel = gap / lmax
    out = {"metric": "precision-form start error vs spectral gaps", "n": n, "nev": int(l.size),
           "fp32_unrefined": {"r0": r0, "residual": acc["residual"], "orthogonality": acc["orthogonality"],
                              "max_eig_err_rel": float(np.max(np.abs(lam.cpu().numpy() - l)) / lmax)},
           "rel_gap": {"min": float(rel.min()), "median": float(np.median(rel)),
                       "p01": float(np.quantile(rel, 0.01))}}
    for name, r in (("fp32", r0), ("bf16_projected", r0 * 2.0 ** 16)):
        out[name] = {"r0": r, "pairs_with_correction_above_0.25": int(np.sum(r / rel > 0.25)),
                     "fraction": float(np.mean(r / rel > 0.25))}
    h.close()
    print(json.dumps(out), flush=True)


def bse_bench(args):
    """--workload bse: the Bethe-Salpeter route (skew_evd_bse: M, Cholesky,
    K = L^T J L, the skew-symmetric solve, back-transformation) on synthetic
    complex blocks of order m = n/2 (n = 10000 by default through --n), all m
    positive eigenpairs.  Flops counted: (1/3) n^3 Cholesky + n^3 for the lower
    half of K + the skew solve's F(n) + 2 n^2 (2 nev) for the triangular solve."""
    import torch
    from paper_1912_04062_amd import skewevd, workloads
    n = args.n if args.n != 16384 else 10000
    m = n // 2
    A, B = workloads.bse_complex(m, 3)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()
    h = skewevd.Handle()
    nev = m
    F = n ** 3 / 3.0 + n ** 3 + useful_flops(n, nev) + 4.0 * n * n * nev
    for _ in range(max(args.warmup, 1)):
        h.bse(Ad, Bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lam, X = h.bse(Ad, Bd)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    # the skew-symmetric part alone, on a matrix of the same order
    K = workloads.random_skew(n, 3)
    Kd = torch.from_numpy(np.ascontiguousarray(K.T)).cuda().t()
    h.solve(Kd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.solve(Kd)
    torch.cuda.synchronize()
    wskew = (time.perf_counter() - t0) / args.steps
    h.close()
    print(json.dumps({"metric": "Bethe-Salpeter route time-to-solution, all positive eigenpairs, TFLOP/s",
                      "value": F / wall / 1e12, "unit": "TFLOP/s", "ms_per_step": wall * 1e3,
                      "steps": args.steps, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"complex BSE blocks A = diag(d) + V V^H / m, B = 0.1 W W^T / m, "
                                             f"m = {m} (order {n}), seed 3, nev = m", "n": n, "m": m,
                                 "flops": F},
                      "skew_solve_ms_same_order": wskew * 1e3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="dense", choices=["dense", "batch", "start", "bse"],
                    help="dense: one matrix of order --n (the headline line); batch: 512 "
                         "uneven matrices through the batched entry point")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--nev", type=int, default=0,
                    help="eigenpairs (0 = n/2, the headline); fewer for a partial-spectrum line")
    ap.add_argument("--reduction", default="two", choices=["two", "one", "complex"],
                    help="two-stage (the headline), the one-stage reduction of Section 2.3.1 "
                         "(FP64; for the one- vs two-stage comparison), or the complex Hermitian "
                         "route on iA (FP64; the complex-arithmetic comparison)")
    ap.add_argument("--all-pairs", action="store_true",
                    help="all n eigenpairs of both signs (the 100 %% case; the other half is a copy)")
    ap.add_argument("--precision", default="both", choices=["fp64", "fp32", "both"])
    ap.add_argument("--check", type=int, default=1, help="untimed accuracy check of each form")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3072)
    ap.add_argument("--autotune", default="both", choices=["0", "1", "both"],
                    help="--workload batch: time the fixed band rule, the autotuned bands, or both")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="MiB copied by one plain device copy before the solves (a known-size "
                         "reference for hardware byte counters); 0 = none")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        # the batched form runs its problems on 16 streams: let the HIP runtime
        # give each its own hardware queue (read when the runtime starts, so
        # before torch initializes the device)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
        batch_bench(args)
        return
    if args.workload == "start":
        start_study(args)
        return
    if args.workload == "bse":
        bse_bench(args)
        return

    import torch
    from paper_1912_04062_amd import skewevd, workloads

    n = args.n
    nev = args.nev if args.nev > 0 else (n + 1) // 2
    nout = n if args.all_pairs else nev
    A = workloads.random_skew(n, 4)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    del A
    if args.copy_calib > 0:
        nel = args.copy_calib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = skewevd.Handle()
    out = (torch.empty(nout, dtype=torch.float64, device="cuda"),
           skewevd.empty_colmajor(n, nout, "cuda"), skewevd.empty_colmajor(n, nout, "cuda"))
    F = useful_flops(n, (n + 1) // 2 if args.all_pairs else nev)
    forms = ["fp64", "fp32"] if args.precision == "both" else [args.precision]
    if args.reduction != "two":
        forms = ["fp64"]            # the one-stage routes are FP64 only
    results = {}
    warm = max(args.warmup, 1)      # at least one untimed run (it also names the dominant kernel)
    for form in forms:
        # untimed runs time every kernel class (the table of kernels_ms) and name
        # the dominant kernel; the timed steps then keep HIP events only around
        # that kernel when it is the stage-2 application (one launch), so that
        # the timers of the many small launches stay out of the timed region
        full = None
        def opts(prof):
            return skewevd.default_opts(form, profile=prof, all_pairs=int(args.all_pairs),
                                        reduction=args.reduction)
        for w in range(warm):
            h.solve(Ad, nev=nev, out=out, opts=opts(1))
            full = h.last_info.as_dict()
        torch.cuda.synchronize()
        kfull = {k: v["ms"] for k, v in full["kernels"].items()}
        prof = 2 if max(kfull, key=kfull.get) == "bt2" else 1
        infos = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            h.solve(Ad, nev=nev, out=out, opts=opts(prof))
            infos.append(h.last_info.as_dict())
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        acc = accuracy(Ad, *out) if args.check else None      # untimed
        results[form] = {"wall": wall, "infos": infos, "accuracy": acc, "kernels_untimed": kfull,
                         "refine_sweeps": infos[-1]["refine_sweeps"]}

    def ok(form):
        a = results[form]["accuracy"]
        return a is None or (a["residual"] <= 1e-13 and a["orthogonality"] <= 1e-13)

    best = min((f for f in forms if ok(f)), key=lambda f: results[f]["wall"], default=forms[0])
    wall = results[best]["wall"]
    infos = results[best]["infos"]
    ms = wall * 1e3
    value = F / wall / 1e12

    # dominant kernel of the reported form: the largest average device time
    stage_avg = {k: float(np.mean([i["ms_stage"][k] for i in infos])) for k in infos[0]["ms_stage"]}
    kern = {k: float(np.mean([i["kernels"][k]["ms"] for i in infos])) for k in infos[0]["kernels"]}
    dom = max(results[best]["kernels_untimed"], key=results[best]["kernels_untimed"].get)
    kinfo = infos[0]["kernels"][dom]
    dtype = "f64" if best == "fp64" else "f32+f64"
    kdtype = "f64" if (best == "fp64" or dom in ("bulge_chase", "tridiag", "refine", "panel_qr")) else "f32"
    if kinfo["bound"] == "hbm":
        achieved = kinfo["bytes"] / (kern[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s"}
    else:
        achieved = kinfo["flops"] / (kern[dom] * 1e-3) / 1e12
        roof = {"bound": kinfo["bound"], "achieved": achieved, "peak": PEAK[kdtype], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_record(dom) if best == "fp64" else None
    roof["kernel"] = dom
    roof["gpu_kernel"] = {"panel_qr": "k_panel_qr", "bulge_chase": "k_bulge_chase", "bt2": "k_bt2_win",
                          "bt1": "k_bt1_w + k_bt1_t + k_bt1_z", "tridiag": "k_bisect + k_invit + orthogonalization",
                          "skew_symm_w": "k_skew_symm + k_gram + k_small + k_wform",
                          "skew_syr2k": "k_skew_syr2k", "refine": "refinement kernels"}.get(dom, dom)
    if args.reduction == "one" and dom == "panel_qr":
        roof["gpu_kernel"] = "k_os_col + k_os_symv + k_os_dots + k_os_w + k_skew_syr2k (one-stage reduction)"
    if args.reduction == "complex" and dom == "panel_qr":
        roof["gpu_kernel"] = "k_h_col + k_h_hemv + k_h_dots + k_h_w + k_her2k (complex Hermitian reduction)"
    roof["launches_per_step"] = kinfo["launches"]
    roof["ms_per_step"] = kern[dom]
    roof["kernels_ms"] = results[best]["kernels_untimed"]   # from an untimed run with every kernel timed
    form_summary = {f: {"ms_per_step": r["wall"] * 1e3, "tflops": F / r["wall"] / 1e12,
                        "refine_sweeps": r["refine_sweeps"], "accuracy": r["accuracy"]}
                    for f, r in results.items()}
    line = {
        "metric": "skew-EVD time-to-solution n=16384, n/2 eigvecs: FP32+refine vs FP64, TFLOP/s",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": warm,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"dense random skew-symmetric A=(B-B^T)/2, B iid N(0,1), seed 4, "
                               f"n={n}, nev={nev}{' (all n pairs)' if args.all_pairs else ''}"
                               f"{ {'two': '', 'one': '; one-stage reduction', 'complex': '; complex Hermitian route on iA'}[args.reduction] }; "
                               f"reported form: {best}",
                   "n": n, "nev": nev, "all_pairs": bool(args.all_pairs), "reduction": args.reduction,
                   "precision": best,
                   "band": infos[0]["band"], "useful_flops": F},
        "forms": form_summary,
        "stages_ms": stage_avg,
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
