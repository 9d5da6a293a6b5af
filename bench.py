"""Benchmark: PALM-KQR fit on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1]

A step is one whole fit (kernel materialisation, RPCholesky preconditioner,
Phase I ADMM, Phase II SSN-ALM to max(eta_kkt, eta_gap) <= 1e-6, final exact
residuals) on a seeded synthetic problem whose X and y are already in device
memory when the timed region starts.

Printed (one JSON line):
  value        whole-job K-apply throughput: bytes of K streamed by all
               K-applies of the timed fits (n^2 * sizeof(entry) per apply)
               divided by the timed wall time, in GB/s;
  ms_per_step  wall time of one fit to relative KKT 1e-6;
  roofline     the dominant kernel (materialised K-apply) timed live with HIP
               events inside the fits: algorithmic bytes n^2*s per launch over
               its average duration, against the 8 TB/s HBM peak;
  cpu_baseline the FP64 oracle's K-apply on a bounded row sample of the same
               K on this host's cores.

The default workload is c1 (n=50000, FP32 K, rank 500).  Other workloads
print one line of the same shape for their own comparison:
  c2     BF16-stored K with FP64 refinement against FP32 K, same problem;
  c2lap  on-the-fly Laplacian K (nothing stored), VALU-bound;
  c3a    nine quantile levels fitted jointly (K V on the matrix cores)
         against nine separate fits;
  c3b    64 uneven problems in one batch against one at a time;
  c4     fit + implicit adjoint of the validation loss (and, with --fd,
         central differences of polished fits).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
METRIC = "K-apply GB/s (% HBM peak) + wall time to rel KKT 1e-6, FP32 vs BF16/batched"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--n", type=int, default=None, help="override the workload size")
    ap.add_argument("--kdtype", default=None, choices=[None, "fp32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU oracle K-apply sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the K-apply shape sweep before the warm-up")
    ap.add_argument("--retune", action="store_true",
                    help="sweep the launch shapes even when paper_2510_07929_amd/tune/<arch>.json holds them")
    ap.add_argument("--tune-out", default=None, help="write the launch shapes in use at the end to this JSON file")
    ap.add_argument("--no-packed", action="store_true", help="single fits: skip the packed-layout comparison")
    ap.add_argument("--no-compare", action="store_true",
                    help="c1: skip the BF16 (c2) and batched (c3a, c3b) comparison legs")
    ap.add_argument("--no-cert", action="store_true", help="single fits: skip the FP64 certificate of the fit")
    ap.add_argument("--certify", action="store_true",
                    help="fit c2 (BF16 and FP32 K), c2lap and c3a at full size and certify each against FP64 "
                         "(one JSON line each; minutes of host time)")
    ap.add_argument("--traffic", default=None,
                    help="counter summary (profiles/*_traffic.md) with the measured HBM bytes per K-apply launch")
    ap.add_argument("--fd", action="store_true", help="c4: also time central differences of the gradient")
    ap.add_argument("--verbose", action="store_true", help="per-iteration solver log on stderr")
    return ap.parse_args()


def _host_ram_gb():
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    return round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:  # pragma: no cover
        pass
    return None


def cpu_baseline(prob, budget_s):
    """The oracle as it stands, timed on this host's cores with the BLAS
    thread count set explicitly: its FP64 K-apply on a row block of the same
    kernel matrix (the line's unit), and whole oracle fits -- the small
    workload at full size with all threads and with one, and this workload at
    a reduced n whose FP64 K fits in a few hundred MB."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import kernel as okernel
    from oracle import solver as osolver
    from paper_2510_07929_amd import inputs

    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        n = prob.n
        rows = max(256, min(n, int(2.0e8 // n)))  # ~1.6 GB of FP64 entries at most
        t0 = time.perf_counter()
        op_block = okernel.kernel_block(prob.X[:rows], prob.X, prob.kernel, prob.gamma)
        t_build = time.perf_counter() - t0
        v = np.random.default_rng(0).standard_normal(n)
        reps, t_apply = 0, 0.0
        while t_apply < max(1.0, budget_s - t_build) and reps < 200:
            t0 = time.perf_counter()
            _ = op_block @ v
            t_apply += time.perf_counter() - t0
            reps += 1
        del op_block
    bytes_per = rows * n * 8.0
    gbs = bytes_per * reps / t_apply / 1e9

    def oracle_fit(name, nn, limit):
        p = inputs.workload(name, n=nn)
        o = osolver.OracleOptions(tol=1e-6, rank=p.rank if p.rank > 0 else 0)
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            r = osolver.fit(p.X, p.y, p.tau, p.lam, p.kernel, p.gamma, o,
                            uniforms=inputs.pivot_uniforms(1024, (sum(map(ord, name)), 0)))
            el = time.perf_counter() - t0
        return {"n": nn, "threads": limit, "s": round(el, 3), "kkt": float(r.kkt["err"]),
                "kernel_applies": int(r.info["kapply"])}

    fits = [oracle_fit("c0", 2000, cores), oracle_fit("c0", 2000, 1)]
    if prob.name != "c0":
        fits.append(oracle_fit(prob.name, min(prob.n, 6000), cores))
    return {
        "value": round(gbs, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"oracle FP64 K-apply (K @ v, materialised FP64 rows) on rows 0..{rows - 1} of the "
                   f"n={n} {prob.kernel} K, {reps} applies; block built by the oracle in {t_build:.1f} s"),
        "full_apply_s_extrapolated": round(t_apply / reps * n / rows, 3),
        "oracle_fits": fits,
        "oracle_fits_note": ("whole oracle fits to max(eta_kkt, eta_gap) <= 1e-6 (dense FP64 Cholesky solves for "
                             "n <= 5000, PCG beyond; active-set polish at the end): the small workload at full size "
                             "with all threads and single-threaded, and this workload at a reduced n (its FP64 K at "
                             "full n would be 8 n^2 bytes)"),
        "blas_threads_set": cores, "affinity_cores": cores, "host_ram_gb": _host_ram_gb(),
    }


def measured_traffic(args, prob, kdtype, layout=0):
    """HBM bytes per launch of the fast K-apply from the committed counter
    summary of this workload (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy
    calibrated), or None when there is none or the kernel source changed
    since the counters were taken."""
    from paper_2510_07929_amd import traffic as tr

    kind = "packed" if layout == 1 else "rows"
    default = os.path.join(ROOT, "profiles", f"kapply_{kind}_{prob.name}_{kdtype}_traffic.md")
    path = (args.traffic if layout == 0 else None) or default
    got = tr.read_summary(path)
    if got is None or got[1] != tr.source_digest(tr.source_for(kind)):
        return None
    return got[0]


def fit_summary(info, st):
    return {
        "status": st, "eta_kkt": info["eta_kkt"], "eta_gap": info["eta_gap"], "obj_p": info["obj_p"],
        "admm_iters": info["admm_iters"], "alm_iters": info["alm_iters"], "newton_iters": info["newton_iters"],
        "admm_pcg_iters": info["admm_pcg_iters"], "pcg_iters": info["pcg_iters"],
        "refinements": info["refinements"], "rank": info["rank_used"],
        "kapply_calls": info["kapply_calls"], "kapply_exact_calls": info["kapply_exact_calls"],
        "t_kbuild_s": round(info["t_kbuild"], 4), "t_precond_s": round(info["t_precond"], 4),
        "t_admm_s": round(info["t_admm"], 4), "t_alm_s": round(info["t_alm"], 4),
        "t_total_s": round(info["t_total"], 4),
        "t_kapply_exact_avg_us": round(info["t_kapply_exact"] / max(info["kapply_exact_calls"], 1) * 1e6, 2),
    }


def base_line(args, prob, dtype, config_extra=None):
    cfg = {
        "workload": f"{prob.name}: {inputs_mod().WORKLOADS[prob.name][1]}",
        "n": prob.n, "p": prob.p, "tau": prob.tau, "lambda": prob.lam, "gamma": prob.gamma,
        "kernel": prob.kernel, "tol": 1e-6,
    }
    cfg.update(config_extra or {})
    return {
        "metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": cfg,
    }


def inputs_mod():
    from paper_2510_07929_amd import inputs

    return inputs


def load_tuning(args):
    """Install the committed launch shapes for this GPU's architecture
    (paper_2510_07929_amd/tune/<arch>.json, written by kqr_tune_save after a
    sweep on that architecture) instead of sweeping; returns the file or None."""
    import torch

    from paper_2510_07929_amd import kqr

    if args.retune or args.no_tune:
        return None
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = os.path.join(ROOT, "paper_2510_07929_amd", "tune", f"{arch}.json")
    if not os.path.exists(path):
        return None
    return os.path.relpath(path, ROOT) if kqr.kqr_tune_load(path) > 0 else None


def timed_fits(args, one_fit):
    import torch

    for _ in range(args.warmup):
        one_fit()
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(one_fit())
    torch.cuda.synchronize()
    return outs, time.perf_counter() - t0


def run_materialised(args, prob, kdtype, tune, layout=0, **extra):
    """Timed single-problem fits with K stored (fp32 or bf16; full rows or the
    symmetric packed tiles); returns (line pieces)."""
    import torch

    from paper_2510_07929_amd import inputs, kqr

    esz = 4 if kdtype == "fp32" else 2
    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    rank = prob.rank if prob.rank > 0 else 0
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
    opts = dict(rank=rank, k_dtype=kqr.KDTYPES[kdtype], kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1,
                verbose=1 if args.verbose else 0, k_layout=layout, **extra)

    last_iterate = {}

    def one_fit():
        alpha, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, uniforms=uni,
                                            out_vz=True, **opts)
        last_iterate.update(alpha=alpha, beta=beta, v=info.pop("v"), z=info.pop("z"))
        return info, st

    tuned = {}
    if tune and args.tuned_from:
        tuned = {"from": args.tuned_from}
        tune = False
    if tune and layout == 1:
        # untimed: pick the packed K-apply shape on this problem's own packed K
        Kp = kqr.kqr_kernel_build_packed(X, prob.kernel, prob.gamma, kdtype)
        modes = [(kqr.KQR_APPLY_FAST, "fast")] + ([(kqr.KQR_APPLY_EXACT, "exact")] if kdtype == "fp32" else [])
        for mode, name in modes:
            tuned[name] = kqr.kqr_autotune_packed(Kp, prob.n, mode, reps=3)["best"]
        del Kp
        torch.cuda.empty_cache()
    if tune and layout == 0:
        # untimed: pick the K-apply tile shapes on this problem's own K
        K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kdtype)
        modes = [(kqr.KQR_APPLY_FAST, "fast")]
        if kdtype == "fp32":
            modes.append((kqr.KQR_APPLY_EXACT, "exact"))
        for mode, name in modes:
            rep = kqr.kqr_autotune_apply(K, mode, reps=3)
            tuned[name] = rep["best"]
        del K
        torch.cuda.empty_cache()
    outs, elapsed = timed_fits(args, one_fit)
    n = prob.n
    kbytes = float(n) * n * esz if layout == 0 else float(kqr.kqr_packed_bytes(n, kdtype))
    nfast = sum(i["kapply_fast_calls"] for i, _ in outs)
    tfast = sum(i["t_kapply_fast"] for i, _ in outs)
    value = nfast * kbytes / elapsed / 1e9
    avg = tfast / max(nfast, 1)
    achieved = kbytes / avg / 1e9 if avg > 0 else 0.0
    traffic = measured_traffic(args, prob, kdtype, layout)
    last, st = outs[-1]
    kname = ("kapply_rows_kernel (fast, materialised %s K)" % kdtype if layout == 0 else
             "kapply_packed_*_kernel + packed_reduce_*_kernel (fast, %s K, symmetric packed tiles)" % kdtype)
    roof = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": kname,
        "avg_launch_us": round(avg * 1e6, 2), "launches": int(nfast),
        "bytes_per_launch": kbytes, "tile_shapes": tuned or "default",
    }
    it = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in last_iterate.items()}
    del X, y
    last_iterate.clear()
    torch.cuda.empty_cache()
    fit = fit_summary(last, st)
    fit["_iterate"] = it
    return value, elapsed / args.steps * 1e3, roof, fit


def error_vs_fp64(prob, fit, kdtype, modes=("fast", "exact")):
    """Error against FP64 of a fit and of one K-apply per precision mode.

    The oracle's FP64 certificate (one pass of FP64 kernel products on the
    host: Section 4 measures at the returned iterate with the exact kernel,
    and a weak-duality bound of the relative objective error) plus the
    relative error ||u - K v|| / ||K v|| of the GPU's K-apply of a random v,
    K v from the same FP64 pass."""
    import numpy as np
    import torch

    from oracle import certify
    from paper_2510_07929_amd import kqr

    it = fit.pop("_iterate")
    t0 = time.perf_counter()
    v = np.random.default_rng(17).standard_normal(prob.n)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kdtype)
    vt = torch.from_numpy(v).to(dev)
    ugpu = {m: kqr.kqr_kernel_apply(vt, K=K, mode=kqr.KQR_APPLY_FAST if m == "fast" else kqr.KQR_APPLY_EXACT)
            .cpu().numpy() for m in modes}
    del K, X, vt
    torch.cuda.empty_cache()
    c = certify.certificate(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, it["alpha"], it["beta"],
                            v=it["v"], z=it["z"], extra=v)
    kv = c["K_extra"][:, 0]
    rel = {f"{m}_{kdtype}_k": float(np.linalg.norm(u - kv) / np.linalg.norm(kv)) for m, u in ugpu.items()}
    return {
        "rel_obj_err_bound": c["rel_obj_err_bound"], "eta_kkt_fp64": c["eta_kkt"], "eta_gap_fp64": c["eta_gap"],
        "eta_p_fp64": c["eta_p"], "eta_d_fp64": c["eta_d"], "eta_c_fp64": c["eta_c"],
        "kapply_rel_err": rel, "n_interior": c["n_interior"],
        "how": ("oracle FP64 certificate on the host (direct-difference FP64 kernel products, oracle/kapply.c): "
                "Section 4 measures at the returned iterate (alpha, v, beta, z) with the exact kernel; "
                "rel_obj_err_bound = (obj_P(alpha, beta) - obj_D(alpha~)) / (1 + |obj_D(alpha~)|) with alpha~ the "
                "feasible projection of alpha (weak duality); K-apply errors ||u - K v|| / ||K v|| of a random v"),
        "seconds": round(time.perf_counter() - t0, 2),
    }


def _leg_args(args):
    import copy

    a = copy.copy(args)
    a.steps, a.warmup = 1, 0
    return a


def compare_bf16_leg(args):
    """The precision workload at full size: BF16-stored K with FP64 refinement
    against FP32-stored K, same problem, same GPU, same KKT target."""
    from paper_2510_07929_amd import inputs

    prob = inputs.workload("c2")
    la = _leg_args(args)
    v16, ms16, roof16, fit16 = run_materialised(la, prob, "bf16", False)
    v32, ms32, roof32, fit32 = run_materialised(la, prob, "fp32", False)
    for f in (fit16, fit32):
        f.pop("_iterate", None)
    return {
        "workload": f"c2: {inputs.WORKLOADS['c2'][1]}", "steps": 1, "warmup": 0,
        "bf16": {"k_storage": "bf16 (inner PCG) + exact FP32 entries recomputed from X (residuals, refinement)",
                 "value": round(v16, 2), "ms_per_step": round(ms16, 3), "roofline": roof16, "fit": fit16},
        "fp32": {"k_storage": "fp32", "value": round(v32, 2), "ms_per_step": round(ms32, 3), "roofline": roof32,
                 "fit": fit32},
        "bf16_speedup": round(ms32 / ms16, 3),
        "error_vs_fp64": "profiles/certificate_c2_c2lap_c3a.md (bench.py --certify)",
    }


def compare_batched_leg(args):
    """Batching at full size: nine quantile levels jointly against nine
    separate fits (c3a), and 64 uneven problems in one batch against one at a
    time (c3b); same GPU, same KKT target."""
    from paper_2510_07929_amd import inputs

    la = _leg_args(args)
    la.no_tune = True
    a = bench_multi_tau(la, inputs.workload("c3a"))
    b = bench_batch(la)
    keep = ("value", "ms_per_step", "roofline", "fit", "compare_separate")
    return {"steps": 1, "warmup": 0,
            "c3a": dict({"workload": a["config"]["workload"]}, **{k: a[k] for k in keep}),
            "c3b": dict({"workload": b["config"]["workload"]}, **{k: b[k] for k in keep})}


def bench_single(args, prob):
    kdtype = args.kdtype or prob.kdtype
    value, ms, roof, fit = run_materialised(args, prob, kdtype, not args.no_tune)
    out = base_line(args, prob, "f32" if kdtype == "fp32" else "bf16", {"k_storage": kdtype, "rank": fit["rank"]})
    out.update(value=round(value, 2), ms_per_step=round(ms, 3), roofline=roof, fit=fit)
    if args.no_cert:
        fit.pop("_iterate", None)
    else:
        out["error_vs_fp64"] = error_vs_fp64(prob, fit, kdtype)
    if not args.no_packed:
        # the same fit with K stored once (symmetric packed tiles): half the bytes per apply
        pv, pms, proof, pfit = run_materialised(args, prob, kdtype, not args.no_tune, layout=1)
        pfit.pop("_iterate", None)
        out["compare_packed"] = {"k_storage": kdtype + ", symmetric packed tiles", "value": round(pv, 2),
                                 "ms_per_step": round(pms, 3), "roofline": proof, "fit": pfit,
                                 "speedup_vs_full": round(ms / pms, 3)}
    if not args.no_compare and prob.name == "c1":
        out["compare_bf16"] = compare_bf16_leg(args)
        out["compare_batched"] = compare_batched_leg(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    return out


def bench_c2(args, prob):
    """BF16-stored K (+ FP64 refinement) against FP32 K on the same problem and GPU."""
    v16, ms16, roof16, fit16 = run_materialised(args, prob, "bf16", not args.no_tune)
    v16c, ms16c, roof16c, fit16c = run_materialised(args, prob, "bf16", False, exact_k=1)
    v32, ms32, roof32, fit32 = run_materialised(args, prob, "fp32", not args.no_tune)
    for f in (fit16, fit16c, fit32):
        f.pop("_iterate", None)
    out = base_line(args, prob, "bf16", {"k_storage": "bf16 (inner) + exact FP32 entries recomputed from X",
                                         "rank": fit16["rank"]})
    out.update(value=round(v16, 2), ms_per_step=round(ms16, 3), roofline=roof16, fit=fit16)
    out["compare_bf16_fp32_copy"] = {"k_storage": "bf16 (inner) + FP32 copy of K (exact applies)",
                                     "value": round(v16c, 2), "ms_per_step": round(ms16c, 3), "roofline": roof16c,
                                     "fit": fit16c, "speedup_vs_fp32": round(ms32 / ms16c, 3)}
    out["compare_fp32"] = {"value": round(v32, 2), "ms_per_step": round(ms32, 3), "roofline": roof32, "fit": fit32,
                           "bf16_speedup": round(ms32 / ms16, 3)}
    if not args.no_packed:
        # K stored once through its symmetry: BF16 tiles for the inner solves
        # and FP32 tiles for the exact applies (22.5 + 45 GB)
        vp, msp, roofp, fitp = run_materialised(args, prob, "bf16", not args.no_tune, layout=1, exact_k=1)
        fitp.pop("_iterate", None)
        out["compare_packed_bf16_fp32_copy"] = {
            "k_storage": "bf16 packed tiles (inner) + FP32 packed tiles (exact applies)", "value": round(vp, 2),
            "ms_per_step": round(msp, 3), "roofline": roofp, "fit": fitp, "speedup_vs_fp32": round(ms32 / msp, 3)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    return out


def bench_otf(args, prob):
    """Nothing stored: every K-apply recomputes the entries (VALU-bound)."""
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))

    def one_fit():
        _, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, uniforms=uni, rank=0,
                                        kmode=kqr.KQR_KMODE_ON_THE_FLY, profile=1, verbose=1 if args.verbose else 0)
        return info, st

    outs, elapsed = timed_fits(args, one_fit)
    n = prob.n
    pairs = float(n) * n
    nfast = sum(i["kapply_fast_calls"] for i, _ in outs)
    tfast = sum(i["t_kapply_fast"] for i, _ in outs)
    avg = tfast / max(nfast, 1)
    # lane operations per evaluated pair of the fast on-the-fly apply.
    # Laplacian (symmetric: each distinct pair once, its entry feeding a row
    # and a column sum): one v_sad_u32 per coordinate of the fixed-point X (p
    # padded to the kernel's bucket), 1 int->float conversion, exp2 (4 ops),
    # 1 scale, 2 FMAs; the algorithmic work is the n (n + 1) / 2 distinct
    # entries.  RBF: p FMAs + 3, exp2 (4 ops), 1 scale, 1 FMA over all n^2.
    if prob.kernel == "laplacian":
        pmax = next(b for b in (8, 12, 16, 20, 24, 32, 48, 64) if prob.p <= b)
        ops = pmax + 8
        work = float(n) * (n + 1) / 2
        kname = ("kapply_otf_l1q_sym_kernel (fast, laplacian, symmetric tiles, fixed-point X, v_sad_u32, "
                 "p=%d padded to %d)" % (prob.p, pmax))
    else:
        ops = prob.p + 3 + 6
        work = pairs
        kname = "kapply_otf_kernel (fast, %s, p=%d)" % (prob.kernel, prob.p)
    peak_pairs = VALU_LANE_OPS / ops
    achieved = work / avg if avg > 0 else 0.0
    last, st = outs[-1]
    out = base_line(args, prob, "f32", {"k_storage": "none (on the fly)", "rank": last["rank_used"]})
    out.update(unit="Gpair/s", value=round(nfast * pairs / elapsed / 1e9, 2), ms_per_step=round(elapsed / args.steps * 1e3, 3))
    out["roofline"] = {
        "bound": "alu", "achieved": round(achieved / 1e9, 2), "peak": round(peak_pairs / 1e9, 2), "unit": "Gpair/s",
        "frac": round(achieved / peak_pairs, 4), "traffic": None,
        "kernel": kname, "avg_launch_us": round(avg * 1e6, 2),
        "launches": int(nfast), "lane_ops_per_pair": ops,
        "peak_note": "non-packed FP32 VALU lane-ops/s of 256 CUs at 2.4 GHz divided by lane ops per pair",
        "work_note": ("achieved counts the distinct entries n (n + 1) / 2 of one apply; value counts n^2 "
                      "pair-equivalents per second of the whole fit") if prob.kernel == "laplacian" else None,
    }
    out["fit"] = fit_summary(last, st)
    return out


def bench_multi_tau(args, prob):
    """Nine quantile levels jointly (one K, K V launches) against nine separate fits."""
    import numpy as np
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    taus = prob.extras["taus"]
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
    kd = args.kdtype or "fp32"
    esz = 4 if kd == "fp32" else 2
    opts = dict(rank=0, k_dtype=kqr.KDTYPES[kd], kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1)

    def joint():
        _, betas, infos, sts = kqr.kqr_fit_multi_tau(X, y, taus, prob.lam, prob.kernel, prob.gamma, uniforms=uni,
                                                     **opts)
        return infos, sts

    tuned = {"from": args.tuned_from} if args.tuned_from else None
    if not args.no_tune and not args.tuned_from:
        # untimed: pick the K V launch shape on this problem's own K
        K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kd)
        tuned = kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_KV, reps=3)["best"]
        del K
        torch.cuda.empty_cache()
    outs, elapsed = timed_fits(args, joint)
    t_sep0 = time.perf_counter()
    sep = [kqr.kqr_fit(X, y, t, prob.lam, prob.kernel, prob.gamma, uniforms=uni, **opts) for t in taus]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t_sep0
    infos, sts = outs[-1]
    nl = infos[0]["kapply_fast_calls"]
    tl = infos[0]["t_kapply_fast"]
    avg = tl / max(nl, 1)
    n = prob.n
    kbytes = float(n) * n * esz
    achieved = kbytes / avg / 1e9 if avg > 0 else 0.0
    out = base_line(args, prob, "f32" if kd == "fp32" else "bf16", {"k_storage": kd, "taus": taus})
    out.update(value=round(nl * kbytes * args.steps / elapsed / 1e9, 2), ms_per_step=round(elapsed / args.steps * 1e3, 3))
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "kernel": ("kv_staged_kernel" if (tuned or {}).get("nld", 0) == 0 else "kv_mfma_kernel")
                  + " (K V, V n x 16, %s K)" % kd, "avg_launch_us": round(avg * 1e6, 2),
        "launches": int(nl), "bytes_per_launch": kbytes, "launch_shape": tuned or "default",
    }
    out["fit"] = {"status": sts, "eta_kkt_max": max(i["eta_kkt"] for i in infos),
                  "eta_gap_max": max(i["eta_gap"] for i in infos),
                  "alm_iters": [i["alm_iters"] for i in infos], "kapply_calls": [i["kapply_calls"] for i in infos]}
    out["compare_separate"] = {
        "ms_total": round(t_sep * 1e3, 3), "status": [s for _, _, _, s in sep],
        "eta_kkt_max": max(i["eta_kkt"] for _, _, i, _ in sep),
        "kapply_calls": int(np.sum([i["kapply_calls"] for _, _, i, _ in sep])),
        "joint_speedup": round(t_sep / (elapsed / args.steps), 3),
    }
    return out


def bench_path(args, prob):
    """A lambda sequence on one K (values coalesced into K V launches) against
    the same values as separate fits."""
    import numpy as np
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    lams = prob.extras["lams"]
    tol = prob.extras["tol"]
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
    kd = args.kdtype or "fp32"
    esz = 4 if kd == "fp32" else 2
    opts = dict(rank=0, k_dtype=kqr.KDTYPES[kd], kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1, tol=tol)

    def path():
        _, betas, infos, sts = kqr.kqr_fit_path(X, y, prob.tau, lams, prob.kernel, prob.gamma, uniforms=uni, **opts)
        return infos, sts

    tuned = {"from": args.tuned_from} if args.tuned_from else None
    if not args.no_tune and not args.tuned_from:
        K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kd)
        tuned = kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_KV, reps=5)["best"]
        kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_FAST, reps=5)
        kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_EXACT, reps=5)
        del K
        torch.cuda.empty_cache()
    outs, elapsed = timed_fits(args, path)
    t_sep0 = time.perf_counter()
    sep = [kqr.kqr_fit(X, y, prob.tau, lam, prob.kernel, prob.gamma, uniforms=uni, **opts) for lam in lams]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t_sep0
    infos, sts = outs[-1]
    nl = infos[0]["kapply_fast_calls"]
    tl = infos[0]["t_kapply_fast"]
    avg = tl / max(nl, 1)
    n = prob.n
    kbytes = float(n) * n * esz
    achieved = kbytes / avg / 1e9 if avg > 0 else 0.0
    out = base_line(args, prob, "f32" if kd == "fp32" else "bf16",
                    {"k_storage": kd, "lambdas": f"{len(lams)} values log-spaced over [{min(lams):g}, {max(lams):g}]",
                     "lambda": None, "tol": tol})
    out.update(value=round(nl * kbytes * args.steps / elapsed / 1e9, 2), ms_per_step=round(elapsed / args.steps * 1e3, 3))
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "kernel": "kv_staged_kernel (K V, V n x 16, %s K)" % kd, "avg_launch_us": round(avg * 1e6, 2),
        "launches": int(nl), "bytes_per_launch": kbytes, "launch_shape": tuned or "default",
    }
    out["fit"] = {"status": sts, "eta_kkt_max": max(i["eta_kkt"] for i in infos),
                  "eta_gap_max": max(i["eta_gap"] for i in infos),
                  "rank": infos[0]["rank_used"],
                  "kapply_calls_total": int(np.sum([i["kapply_calls"] for i in infos])),
                  "alm_iters": [i["alm_iters"] for i in infos], "n_interior": [i["n_interior"] for i in infos]}
    out["compare_separate"] = {
        "ms_total": round(t_sep * 1e3, 3), "status": [s for _, _, _, s in sep],
        "eta_kkt_max": max(i["eta_kkt"] for _, _, i, _ in sep),
        "kapply_calls": int(np.sum([i["kapply_calls"] for _, _, i, _ in sep])),
        "joint_speedup": round(t_sep / (elapsed / args.steps), 3),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    return out


def bench_linear(args, prob):
    """The lambda sequence of Table 2's linear-kernel rows: K = X X^T applied in
    factored form (O(n p) per apply), X as the preconditioner factor; the
    sequence as one call against the same values as separate fits."""
    import numpy as np
    import torch

    from paper_2510_07929_amd import kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    lams = prob.extras["lams"]
    tol = prob.extras["tol"]
    opts = dict(tol=tol, profile=1)

    def path():
        _, betas, infos, sts = kqr.kqr_fit_path(X, y, prob.tau, lams, "linear", 1.0, **opts)
        return infos, sts

    outs, elapsed = timed_fits(args, path)
    t0 = time.perf_counter()
    sep = [kqr.kqr_fit(X, y, prob.tau, lam, "linear", 1.0, **opts) for lam in lams]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    infos, sts = outs[-1]
    n, p = prob.n, prob.p
    napp = sum(i["kapply_fast_calls"] for i in infos)
    tapp = sum(i["t_kapply_fast"] for i in infos)
    avg = tapp / max(napp, 1)
    abytes = 2.0 * n * p * 4 + 2.0 * n * 8  # X read twice, v read, u written
    achieved = abytes / avg / 1e9 if avg > 0 else 0.0
    out = base_line(args, prob, "f64", {"k_storage": "none (factored X X^T)", "lambda": None, "tol": tol,
                                        "lambdas": f"{len(lams)} values log-spaced over [{min(lams):g}, {max(lams):g}]"})
    out.update(value=None, ms_per_step=round(elapsed / args.steps * 1e3, 3))
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": None,
        "kernel": "lin_xtv_kernel + finalize + lin_xt_kernel (X (X^T v), latency-bound at this size)",
        "avg_launch_us": round(avg * 1e6, 2), "launches": int(napp), "bytes_per_launch": abytes,
    }
    out["fit"] = {"status": sts, "eta_kkt_max": max(i["eta_kkt"] for i in infos),
                  "eta_gap_max": max(i["eta_gap"] for i in infos), "rank": infos[0]["rank_used"],
                  "kapply_calls_total": int(np.sum([i["kapply_calls"] for i in infos])),
                  "pcg_iters_total": int(np.sum([i["pcg_iters"] + i["admm_pcg_iters"] for i in infos])),
                  "alm_iters": [i["alm_iters"] for i in infos], "n_interior": [i["n_interior"] for i in infos]}
    out["compare_separate"] = {"ms_total": round(t_sep * 1e3, 3), "status": [s for _, _, _, s in sep],
                               "joint_speedup": round(t_sep / (elapsed / args.steps), 3)}
    out["note"] = "value is null: the linear kernel's apply is O(n p); the line reports the time of the sequence"
    return out


def bench_ablation(args, prob):
    """The two-phase method against each phase alone and against plain CG
    (no preconditioner), on one problem, with per-iteration traces."""
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    tol = prob.extras["tol"]
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
    variants = {
        "palm": {},
        "admm_alone": dict(admm_tol=tol, admm_max_iter=1000, alm_max_iter=0),
        "ssn_alm_alone": dict(admm_max_iter=0, alm_max_iter=1000),
        "palm_plain_cg": dict(rank=-1),
    }
    base = dict(tol=tol, rank=0, kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1)
    res = {}
    t_palm = None
    for name, kw in variants.items():
        opts = dict(base, **kw)
        for _ in range(args.warmup if name == "palm" else 0):
            kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, uniforms=uni, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = args.steps if name == "palm" else 1
        for _ in range(reps):
            _, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, uniforms=uni,
                                            trace=4000, **opts)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        if name == "palm":
            t_palm = el
        tr = info.pop("trace")
        step = max(1, len(tr) // 60)
        res[name] = {
            "s": round(el, 4), "status": st, "err": max(info["eta_kkt"], info["eta_gap"]),
            "admm_iters": info["admm_iters"], "alm_iters": info["alm_iters"], "newton_iters": info["newton_iters"],
            "pcg_iters": info["admm_pcg_iters"] + info["pcg_iters"], "kapply_calls": info["kapply_calls"],
            "rank": info["rank_used"],
            "trace_every": step,
            "trace": [[int(r[0]), int(r[1]), float("%.3e" % r[2]), round(float(r[3]), 4)] for r in tr[::step]]
                     + ([[int(tr[-1][0]), int(tr[-1][1]), float("%.3e" % tr[-1][2]), round(float(tr[-1][3]), 4)]]
                        if len(tr) and (len(tr) - 1) % step else []),
        }
    out = base_line(args, prob, "f32", {"k_storage": "fp32", "tol": tol})
    out.update(value=None, ms_per_step=round(t_palm * 1e3, 3))
    out["ablation"] = res
    out["note"] = ("value is null: this line compares solver variants on one problem; K-apply rates are "
                   "on the c1 line")
    return out


def bench_batch(args):
    """64 uneven problems in one batched fit against the same fits one at a time."""
    import numpy as np
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    probs = inputs.uneven_batch()
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    taus = [p.tau for p in probs]
    lams = [p.lam for p in probs]
    gams = [p.gamma for p in probs]
    opts = dict(rank=0, kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1)

    def batch():
        _, betas, infos, sts = kqr.kqr_fit_batch(Xs, ys, taus, lams, gams, "rbf", **opts)
        return infos, sts

    outs, elapsed = timed_fits(args, batch)
    t0 = time.perf_counter()
    sep = [kqr.kqr_fit(Xs[i], ys[i], taus[i], lams[i], "rbf", gams[i], **opts) for i in range(len(probs))]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    infos, sts = outs[-1]
    nl = infos[0]["kapply_fast_calls"]
    tl = infos[0]["t_kapply_fast"]
    ns = [p.n for p in probs]
    out = {
        "metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3b: 64 uneven problems, n_i ~ U{500..8000}, p=10, RBF gamma=1/p, tau=0.5, "
                               "lambda_i=1e-3 n_i", "n_min": min(ns), "n_max": max(ns), "sum_n2": int(sum(n * n for n in ns))},
    }
    kapply_sep = int(np.sum([i["kapply_calls"] for _, _, i, _ in sep]))
    # every apply of a problem streams that problem's K once; the batched launches carry them all
    per_problem_calls = [i["kapply_calls"] for i in infos]
    streamed = float(sum(c * p.n * p.n * 4 for c, p in zip(per_problem_calls, probs)))
    out["value"] = round(streamed / (elapsed / args.steps) / 1e9, 2)
    out["roofline"] = {
        "bound": "hbm", "achieved": round(streamed / max(tl, 1e-12) / 1e9, 1) if tl > 0 else None, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(streamed / max(tl, 1e-12) / 1e9 / HBM_PEAK_GBS, 4) if tl > 0 else None,
        "traffic": None, "kernel": "kapply_problems_queue_kernel (persistent launch; workgroups take (problem, 32-row block) items from a queue)",
        "launches": int(nl), "avg_launch_us": round(tl / max(nl, 1) * 1e6, 2),
        "note": "achieved = bytes of every problem's K over all its applies / device time of the batched launches; "
                "K matrices of up to 256 MB sit partly in the 256 MB last-level cache",
    }
    out["fit"] = {"status_ok": int(sum(1 for s in sts if s == 0)), "eta_kkt_max": max(i["eta_kkt"] for i in infos),
                  "eta_gap_max": max(i["eta_gap"] for i in infos), "kapply_calls_total": int(sum(per_problem_calls))}
    out["compare_separate"] = {"ms_total": round(t_sep * 1e3, 3), "kapply_calls_total": kapply_sep,
                               "batch_speedup": round(t_sep / (elapsed / args.steps), 3)}
    return out


def bench_grad(args, prob):
    """Fit + implicit adjoint of the validation check loss (c4)."""
    import numpy as np
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    Xv = torch.from_numpy(prob.extras["Xval"]).to(dev)
    yv = torch.from_numpy(prob.extras["yval"]).to(dev)
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
    opts = dict(rank=0, kmode=kqr.KQR_KMODE_MATERIALIZE, profile=1, uniforms=uni)

    def grad_at(gam, lam):
        return kqr.kqr_fit_grad(X, y, prob.tau, lam, prob.kernel, gam, Xv, yv, **opts)

    def step():
        return grad_at(prob.gamma, prob.lam)

    outs, elapsed = timed_fits(args, step)
    t0 = time.perf_counter()
    _, _, info_fit, st_fit = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, **opts)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    alpha, beta, J, (dg, dl), m, pol, info, st = outs[-1]
    n = prob.n
    out = base_line(args, prob, "f32", {"k_storage": "fp32", "nval": int(Xv.shape[0])})
    out.update(unit="GB/s", ms_per_step=round(elapsed / args.steps * 1e3, 3))
    nfast, tfast = info["kapply_fast_calls"], info["t_kapply_fast"]
    kbytes = float(n) * n * 4
    avg = tfast / max(nfast, 1)
    out["value"] = round(nfast * kbytes / (elapsed / args.steps) / 1e9, 2)
    out["roofline"] = {"bound": "hbm", "achieved": round(kbytes / avg / 1e9, 1) if avg > 0 else None,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(kbytes / avg / 1e9 / HBM_PEAK_GBS, 4)
                       if avg > 0 else None, "traffic": None, "kernel": "kapply_rows_kernel (fit part)",
                       "avg_launch_us": round(avg * 1e6, 2), "launches": int(nfast)}
    out["grad"] = {"J": J, "dJ_dlog_gamma": dg, "dJ_dlog_lambda": dl, "n_interior": m, "polished": pol,
                   "status": st, "ms_fit_only": round(t_fit * 1e3, 3),
                   "ms_adjoint": round(elapsed / args.steps * 1e3 - t_fit * 1e3, 3)}
    if args.fd:
        # Central differences of polished fits.  The loss is piecewise smooth:
        # an interval that crosses a kink (a validation residual changing sign
        # or a coefficient entering or leaving the interior set) is flagged,
        # and smaller steps are tried until one is kink-free.
        t0 = time.perf_counter()

        def probe(gam, lam):
            a, b, J, _, _, pol, _, _ = grad_at(gam, lam)
            f = kqr.kqr_predict(X, a, b, lam, prob.kernel, gam, Xv)
            sgn = torch.sign(yv - f).cpu().numpy()
            ac = a.cpu().numpy()
            E = (ac > prob.tau - 1.0) & (ac < prob.tau)
            return J, sgn, E, pol

        J0, s0, E0, _ = probe(prob.gamma, prob.lam)
        fds = []
        for h in (1e-4, 1e-5, 1e-6):
            row = {"h": h}
            for name, g_an in (("gamma", dg), ("lambda", dl)):
                vals, kink, pols = [], False, True
                for sg in (1, -1):
                    gam = prob.gamma * math.exp(sg * h) if name == "gamma" else prob.gamma
                    lam = prob.lam * math.exp(sg * h) if name == "lambda" else prob.lam
                    J, s, E, pol = probe(gam, lam)
                    kink |= not (np.array_equal(s, s0) and np.array_equal(E, E0))
                    pols &= pol
                    vals.append(J)
                fd = (vals[0] - vals[1]) / (2 * h)
                row[name] = {"fd": fd, "rel": abs(fd - g_an) / max(abs(g_an), 1e-300), "kink": bool(kink),
                             "polished": bool(pols)}
            fds.append(row)
            if not (row["gamma"]["kink"] or row["lambda"]["kink"]):
                break
        out["grad"]["fd"] = {"steps": fds, "seconds": round(time.perf_counter() - t0, 3)}
    return out


def bench_certify(args):
    """Full-size fits of the precision and batching workloads, each certified
    against FP64 on the host (oracle.certify); one JSON line per workload."""
    import numpy as np
    import torch

    from oracle import certify
    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    lines = []

    def progress(done, rows):  # the FP64 passes take minutes at these sizes
        print(f"[certify] FP64 kernel products: {done}/{rows} rows", file=sys.stderr, flush=True)

    def apply_errors(prob, modes):
        """||u - K v|| / ||K v|| of one GPU K-apply per mode; K v in FP64 on the host."""
        v = np.random.default_rng(17).standard_normal(prob.n)
        X = torch.from_numpy(prob.X).to(dev)
        vt = torch.from_numpy(v).to(dev)
        us = {}
        for name, kd, mode in modes:
            if kd is None:
                u = kqr.kqr_kernel_apply(vt, X=X, kernel=prob.kernel, gamma=prob.gamma, mode=mode)
            else:
                K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kd)
                u = kqr.kqr_kernel_apply(vt, K=K, mode=mode)
                del K
            us[name] = u.cpu().numpy()
            torch.cuda.empty_cache()
        return v, us

    def one(prob, label, **opts):
        X = torch.from_numpy(prob.X).to(dev)
        y = torch.from_numpy(prob.y).to(dev)
        uni = inputs.pivot_uniforms(1024, (sum(map(ord, prob.name)), 0))
        t0 = time.perf_counter()
        alpha, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, uniforms=uni,
                                            out_vz=True, **opts)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t0
        it = dict(alpha=alpha.cpu().numpy(), v=info.pop("v").cpu().numpy(), z=info.pop("z").cpu().numpy())
        del X, y, alpha
        torch.cuda.empty_cache()
        return dict(label=label, status=st, t_fit_s=round(t_fit, 3), gpu_eta_kkt=info["eta_kkt"],
                    gpu_eta_gap=info["eta_gap"], rank=info["rank_used"], kapply_calls=info["kapply_calls"]), it, beta

    def certified(prob, label, modes, **opts):
        row, it, beta = one(prob, label, **opts)
        v, us = apply_errors(prob, modes)
        t0 = time.perf_counter()
        c = certify.certificate(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, it["alpha"], beta,
                                v=it["v"], z=it["z"], extra=v, progress=progress)
        kv = c["K_extra"][:, 0]
        row.update(eta_kkt_fp64=c["eta_kkt"], eta_gap_fp64=c["eta_gap"], eta_p_fp64=c["eta_p"],
                   eta_d_fp64=c["eta_d"], eta_c_fp64=c["eta_c"], rel_obj_err_bound=c["rel_obj_err_bound"],
                   n_interior=c["n_interior"],
                   kapply_rel_err={k: float(np.linalg.norm(u - kv) / np.linalg.norm(kv)) for k, u in us.items()},
                   t_certificate_s=round(time.perf_counter() - t0, 1))
        return row

    c2 = inputs.workload("c2")
    F, E = kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT
    for kd in ("bf16", "fp32"):
        modes = [(f"fast_{kd}_k", kd, F)] + ([("exact_fp32_k", "fp32", E)] if kd == "fp32" else
                                             [("exact_on_the_fly", None, E)])
        lines.append(dict(workload="c2", **certified(c2, f"{kd} K", modes, rank=0, k_dtype=kqr.KDTYPES[kd],
                                                     kmode=kqr.KQR_KMODE_MATERIALIZE)))
        print(json.dumps(lines[-1]), flush=True)
    lap = inputs.workload("c2lap")
    lines.append(dict(workload="c2lap", **certified(lap, "on the fly", [("fast_on_the_fly", None, F),
                                                                          ("exact_on_the_fly", None, E)],
                                                     rank=0, kmode=kqr.KQR_KMODE_ON_THE_FLY)))
    print(json.dumps(lines[-1]), flush=True)
    c3 = inputs.workload("c3a")
    X = torch.from_numpy(c3.X).to(dev)
    y = torch.from_numpy(c3.y).to(dev)
    taus = c3.extras["taus"]
    uni = inputs.pivot_uniforms(1024, (sum(map(ord, c3.name)), 0))
    t0 = time.perf_counter()
    A, betas, infos, sts = kqr.kqr_fit_multi_tau(X, y, taus, c3.lam, c3.kernel, c3.gamma, uniforms=uni, rank=0,
                                                 kmode=kqr.KQR_KMODE_MATERIALIZE)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    A = A.cpu().numpy()
    del X, y
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    cs = certify.certificate_levels(c3.X, c3.y, taus, c3.lam, c3.kernel, c3.gamma, list(A), list(betas),
                                    progress=progress)
    lines.append(dict(workload="c3a", label="nine levels jointly (FP32 K, K V)", t_fit_s=round(t_fit, 3),
                      status=sts, t_certificate_s=round(time.perf_counter() - t0, 1),
                      levels=[dict(tau=c["tau"], gpu_eta_kkt=i["eta_kkt"], gpu_eta_gap=i["eta_gap"],
                                   res_eta_d_fp64=c["res_eta_d"], res_eta_c_fp64=c["res_eta_c"],
                                   res_eta_gap_fp64=c["res_eta_gap"], rel_obj_err_bound=c["rel_obj_err_bound"],
                                   n_interior=c["n_interior"]) for c, i in zip(cs, infos)]))
    print(json.dumps(lines[-1]), flush=True)
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    from paper_2510_07929_amd import inputs

    w = args.workload
    args.tuned_from = load_tuning(args)
    if args.certify:
        bench_certify(args)
        return
    if w == "c3b":
        out = bench_batch(args)
    else:
        prob = inputs.workload(w, n=args.n)
        if w == "c2" and args.kdtype is None:
            out = bench_c2(args, prob)
        elif w == "c2lap":
            out = bench_otf(args, prob)
        elif w == "c3a":
            out = bench_multi_tau(args, prob)
        elif w == "c4":
            out = bench_grad(args, prob)
        elif w == "path":
            out = bench_path(args, prob)
        elif w == "ablation":
            out = bench_ablation(args, prob)
        elif w == "linear":
            out = bench_linear(args, prob)
        else:
            out = bench_single(args, prob)
    if args.tune_out:
        from paper_2510_07929_amd import kqr

        out["tune_entries_written"] = kqr.kqr_tune_save(args.tune_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
