"""HBM traffic of a kernel from rocprofv3 counters, calibrated by a plain copy.

    python -m paper_2510_07929_amd.traffic copy [--gib 4]
        device-to-device copy of a known size (the calibration dispatch);
    python -m paper_2510_07929_amd.traffic summarize --kernel NAME \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --out FILE.md
        reads the counter CSVs of four rocprofv3 --pmc runs (FETCH_SIZE and
        WRITE_SIZE, each for the measured command and for the copy) and writes
        the per-dispatch HBM bytes of the kernel, each counter scaled by what
        it reads for the copy of known size.

`bench.py` reports the summary's figure as roofline.traffic when the
summary's recorded source digest matches the current kernel source
(`--layout rows`: the materialised section of csrc/kmat.hip; `--layout
packed`: csrc/kpacked.hip).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kmat.hip")
PACKED_SOURCE = os.path.join(HERE, "csrc", "kpacked.hip")


RULE = "// ================================================================= "
SECTIONS = {
    KERNEL_SOURCE: (RULE + "materialised K-apply", RULE + "on-the-fly K-apply"),
    PACKED_SOURCE: (RULE + "apply", RULE + "one row"),
}


def source_digest(path: str = KERNEL_SOURCE) -> str:
    """Digest of a K-apply's source: the section of kmat.hip or kpacked.hip
    that holds its kernels, shape table and launcher."""
    with open(path) as f:
        text = f.read()
    begin, end = SECTIONS[path]
    a, b = text.find(begin + "\n"), text.find(end + "\n")
    if a < 0 or b <= a:
        raise ValueError(f"K-apply section markers not found in {path}")
    return hashlib.sha256(text[a:b].encode()).hexdigest()[:16]


def source_for(layout: str) -> str:
    return PACKED_SOURCE if layout == "packed" else KERNEL_SOURCE


def copy_once(gib: float, reps: int) -> None:
    import torch

    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes x {reps}", flush=True)


def _rows(path_dir: str):
    files = glob.glob(os.path.join(path_dir, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection csv under {path_dir}")
    for fn in files:
        with open(fn, newline="") as f:
            yield from csv.DictReader(f)


def per_dispatch(path_dir: str, counter: str, name_re: str):
    """{dispatch id: counter value} for dispatches whose kernel name matches."""
    rx = re.compile(name_re)
    out = {}
    for r in _rows(path_dir):
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
        cname = r.get("Counter_Name") or r.get("Counter-Name") or ""
        if cname != counter or not rx.search(name):
            continue
        did = r.get("Dispatch_Id") or r.get("Dispatch-Id") or str(len(out))
        out[did] = out.get(did, 0.0) + float(r.get("Counter_Value") or r.get("Counter-Value") or 0.0)
    return out


def summarize(args) -> None:
    fetch = per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    write = per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    cfetch = per_dispatch(args.copy_fetch, "FETCH_SIZE", args.copy_kernel)
    cwrite = per_dispatch(args.copy_write, "WRITE_SIZE", args.copy_kernel)
    if not (fetch and write and cfetch and cwrite):
        raise SystemExit(f"missing dispatches: {len(fetch)} {len(write)} {len(cfetch)} {len(cwrite)}")
    copy_bytes = args.copy_bytes
    kf = sum(cfetch.values()) / len(cfetch)  # KiB per copy dispatch
    kw = sum(cwrite.values()) / len(cwrite)
    f_fetch = copy_bytes / (kf * 1024.0)
    f_write = copy_bytes / (kw * 1024.0)
    mf = sum(fetch.values()) / len(fetch)
    mw = sum(write.values()) / len(write)
    rd = mf * 1024.0 * f_fetch
    wr = mw * 1024.0 * f_write
    lines = [
        f"# HBM traffic per dispatch: {args.title}",
        "",
        "Commands (from the repository root, TMPDIR=/tmp, one counter per run):",
        "```",
        *args.command,
        "```",
        "",
        f"kernel name pattern: `{args.kernel}`; {len(fetch)} dispatches (FETCH_SIZE), {len(write)} (WRITE_SIZE)",
        f"copy calibration: `{args.copy_kernel}`, {copy_bytes:.6g} bytes read and written per dispatch;",
        f"FETCH_SIZE {kf:.6g} KiB -> factor {f_fetch:.4f}; WRITE_SIZE {kw:.6g} KiB -> factor {f_write:.4f}",
        "",
        f"FETCH_SIZE mean {mf:.6g} KiB -> {rd:.6g} bytes read per dispatch",
        f"WRITE_SIZE mean {mw:.6g} KiB -> {wr:.6g} bytes written per dispatch",
        f"algorithmic bytes per dispatch: {args.algorithmic:.6g}",
        "",
        f"traffic_bytes_per_launch: {rd + wr:.6g}",
        f"source_digest: {source_digest(source_for(args.layout))}",
    ]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_summary(path: str):
    """(bytes per launch, digest) from a summary written by `summarize`, or None."""
    if not os.path.exists(path):
        return None
    val = dig = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_bytes_per_launch:"):
                val = float(line.split(":", 1)[1])
            elif line.startswith("source_digest:"):
                dig = line.split(":", 1)[1].strip()
    if val is None or dig is None:
        return None
    return val, dig


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--gib", type=float, default=4.0)
    c.add_argument("--reps", type=int, default=3)
    s = sub.add_parser("summarize")
    s.add_argument("--kernel", required=True, help="regular expression on the kernel name")
    s.add_argument("--copy-kernel", default="copyBuffer|copy", help="regular expression for the copy dispatch")
    s.add_argument("--copy-bytes", type=float, required=True)
    s.add_argument("--algorithmic", type=float, required=True)
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--copy-fetch", required=True)
    s.add_argument("--copy-write", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--out", required=True)
    s.add_argument("--layout", default="rows", choices=["rows", "packed"],
                   help="which K-apply source the summary is tied to")
    args = ap.parse_args(argv)
    if args.cmd == "copy":
        copy_once(args.gib, args.reps)
    else:
        summarize(args)


if __name__ == "__main__":
    sys.exit(main())
