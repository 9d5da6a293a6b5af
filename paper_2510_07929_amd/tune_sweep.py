"""Launch-shape sweep for this GPU's architecture -> paper_2510_07929_amd/tune/<arch>.json.

    python -m paper_2510_07929_amd.tune_sweep [--out FILE]

Runs every autotuner of the library on the seeded inputs of the benchmark
workloads and writes the installed shapes with kqr_tune_save:

* materialised K-apply, fast and exact: FP32 K at n = 50,000 (p = 20) and at
  n = 150,000 (p = 30), BF16 K (fast) at n = 150,000;
* symmetric packed K-apply, fast and exact: FP32 at n = 50,000;
* K V (up to 16 right-hand sides): FP32 K at n = 20,000 (the lambda path
  of Section 4.1) and n = 100,000 (the single-vector shapes of those sizes
  share the size classes of n = 50,000 and 150,000, swept above);
* on-the-fly square applies (strip per size class, slice target): the
  Laplacian at n = 300,000 (fast and exact), then the RBF with p = 30 at
  n = 150,000 (exact, the residuals of the BF16 fits).

bench.py and any process started with KQR_TUNE_FILE=<file> load the file
instead of sweeping.  Needs about 100 GB of device memory at its peak (the
FP32 K at n = 150,000); a few minutes on one MI355X.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> None:
    import torch

    from paper_2510_07929_amd import inputs, kqr

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="output file (default: paper_2510_07929_amd/tune/<arch>.json)")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = a.out or os.path.join(ROOT, "paper_2510_07929_amd", "tune", f"{arch}.json")
    F, E, KV = kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT, kqr.KQR_APPLY_KV

    def say(*m):
        print("[sweep]", *m, flush=True)

    def best(rep):
        return rep.get("best")

    # materialised K-apply
    for name, kd, modes in (("c1", "fp32", (F, E)), ("c2", "fp32", (F, E)), ("c2", "bf16", (F,))):
        prob = inputs.workload(name)
        X = torch.from_numpy(prob.X).to(dev)
        K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, kd)
        for m in modes:
            say(f"apply {name} {kd} mode {m}:", best(kqr.kqr_autotune_apply(K, m, reps=a.reps)))
        if name == "c1" and kd == "fp32":
            del K
            torch.cuda.empty_cache()
            Kp = kqr.kqr_kernel_build_packed(X, prob.kernel, prob.gamma, kd)
            for m in (F, E):
                say(f"packed {name} {kd} mode {m}:", best(kqr.kqr_autotune_packed(Kp, prob.n, m, reps=a.reps)))
            del Kp
        else:
            del K
        del X
        torch.cuda.empty_cache()
    # K V at the lambda-path and joint-level sizes
    for label, prob in (("path", inputs.workload("path")), ("c3a", inputs.workload("c3a"))):
        X = torch.from_numpy(prob.X).to(dev)
        K = kqr.kqr_kernel_build(X, prob.kernel, prob.gamma, "fp32")
        say(f"kv {label}:", best(kqr.kqr_autotune_apply(K, KV, reps=a.reps)))
        del K, X
        torch.cuda.empty_cache()
    # on-the-fly square applies
    for name, modes in (("c2lap", (F, E)), ("c2", (E,))):  # one entry per size class: the RBF's last
        prob = inputs.workload(name)
        X = torch.from_numpy(prob.X).to(dev)
        for m in modes:
            say(f"otf {name} mode {m}:", best(kqr.kqr_autotune_otf(X, prob.kernel, prob.gamma, m, reps=a.reps)))
        del X
        torch.cuda.empty_cache()
    say("wrote", kqr.kqr_tune_save(out), "entries to", out)


if __name__ == "__main__":
    main()
