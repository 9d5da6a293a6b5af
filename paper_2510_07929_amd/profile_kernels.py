"""Counter collection for the compute-bound kernels, and its summary.

    python -m paper_2510_07929_amd.profile_kernels run
        launches each kernel of interest twice on seeded inputs: the K build
        (n = 50,000 FP32 and n = 150,000 BF16), and the on-the-fly square
        apply K(X, X) v, fast and exact, for the RBF at n = 150,000, p = 30
        (BF16x3 Gram), the RBF at n = 100,000, p = 8 (FP32 Gram) and the
        Laplacian at n = 300,000, p = 30 (fixed point);
    python -m paper_2510_07929_amd.profile_kernels batch
        one warm-up and one timed batched fit of the 64 uneven problems
        (n_i in [500, 8000], p = 10), then the same problems one at a time;
        prints the wall times;
    python -m paper_2510_07929_amd.profile_kernels summarize --pmc DIR [DIR ...] --out FILE.md
        reads the counter CSVs of rocprofv3 --pmc runs of `run` and writes a
        per-kernel table (averages over its dispatches).

Run under rocprofv3, one pass per counter group, e.g.
    rocprofv3 --pmc MfmaUtil VALUBusy OccupancyPercent LdsBankConflict -d D1 -o run \\
        --output-format csv -- python3 -m paper_2510_07929_amd.profile_kernels run
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys


def run() -> None:
    import numpy as np
    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    print("[profile] K build", flush=True)
    for name, kd in (("c1", "fp32"), ("c2", "bf16")):
        prob = inputs.workload(name)
        X = torch.from_numpy(prob.X).to(dev)
        for _ in range(2):
            K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kd)
            torch.cuda.synchronize()
            del K
        torch.cuda.empty_cache()
    print("[profile] on-the-fly applies", flush=True)
    for n, p, kind in ((150000, 30, "rbf"), (100000, 8, "rbf"), (300000, 30, "laplacian")):
        X, _ = inputs.additive(n, p, (5, n))
        Xt = torch.from_numpy(X).to(dev)
        v = torch.from_numpy(np.random.default_rng(0).standard_normal(n)).to(dev)
        for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
            for _ in range(2):
                kqr.kqr_kernel_apply(v, X=Xt, kernel=kind, gamma=1.0 / p, mode=mode)
        torch.cuda.synchronize()
    print("[profile] done", flush=True)


def batch() -> None:
    import time

    import torch

    from paper_2510_07929_amd import inputs, kqr

    dev = torch.device("cuda:0")
    probs = inputs.uneven_batch()
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    args = ([p.tau for p in probs], [p.lam for p in probs], [p.gamma for p in probs], "rbf")
    opts = dict(rank=0, kmode=kqr.KQR_KMODE_MATERIALIZE)
    for label in ("warm-up", "timed"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, infos, sts = kqr.kqr_fit_batch(Xs, ys, *args, **opts)
        torch.cuda.synchronize()
        print(f"[profile] batch {label}: {time.perf_counter() - t0:.3f} s, "
              f"{sum(1 for s in sts if s == 0)}/{len(sts)} converged", flush=True)
    t0 = time.perf_counter()
    for i in range(len(probs)):
        kqr.kqr_fit(Xs[i], ys[i], args[0][i], args[1][i], "rbf", args[2][i], **opts)
    torch.cuda.synchronize()
    print(f"[profile] one at a time: {time.perf_counter() - t0:.3f} s", flush=True)


def summarize(dirs, out: str, cmd: str) -> None:
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    for d in dirs:
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True):
            with open(fn, newline="") as f:
                for r in csv.DictReader(f):
                    k = r["Kernel_Name"].split("(")[0].replace("void ", "")
                    agg[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
                    meta[k] = (r["VGPR_Count"], r["Accum_VGPR_Count"], r["LDS_Block_Size"])
    keys = sorted({c for v in agg.values() for c in v})
    lines = ["# Counters of the compute-bound kernels", "",
             "Averages over each kernel's dispatches (two per kernel and mode).", "",
             "Command (one rocprofv3 pass per counter group, in its own output folder):", "", "```", cmd, "```", "",
             "| kernel | VGPR | AGPR | LDS bytes | " + " | ".join(keys) + " |",
             "|---|---|---|---|" + "---|" * len(keys)]
    for k in sorted(agg):
        if not any(s in k for s in ("kbuild_b3", "otf_mfma", "otf_l1q", "kbuild_kernel")):
            continue
        vals = [agg[k].get(c) for c in keys]
        cells = ["%.4g" % (sum(v) / len(v)) if v else "" for v in vals]
        vg, ag, lds = meta[k]
        lines.append(f"| `{k}` | {vg} | {ag} | {lds} | " + " | ".join(cells) + " |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}")


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("run")
    sub.add_parser("batch")
    s = sub.add_parser("summarize")
    s.add_argument("--pmc", nargs="+", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", default="", help="the rocprofv3 command lines, for the summary's header")
    a = ap.parse_args()
    if a.cmd == "run":
        run()
    elif a.cmd == "batch":
        batch()
    else:
        summarize(a.pmc, a.out, a.command)


if __name__ == "__main__":
    sys.exit(main())
