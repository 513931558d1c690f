"""Profiling helpers around rocprofv3 (measurement tooling, not on the solve path).

  python -m paper_2107_00820_amd.profiling copy [--mib 1024] [--reps 3]
      a plain device-to-device copy of known size (the calibration kernel of
      the HBM traffic counters).
  python -m paper_2107_00820_amd.profiling stats DIR OUT.md --title T --cmd C
      summarises the kernel trace CSV that `rocprofv3 --kernel-trace --stats
      --output-format csv -d DIR` wrote.
  python -m paper_2107_00820_amd.profiling traffic --fetch D1 --write D2 --copy-fetch D3
      --copy-write D4 --copy-bytes N --kernel REGEX --out OUT.json --cmd C
      per-launch FETCH_SIZE / WRITE_SIZE of the kernels matching REGEX (from
      two `--pmc` runs), with the factor measured on the copy kernel
      (known bytes / counted bytes), keyed by the exact kernel name and stamped
      with a hash of the kernel sources so a changed kernel invalidates it.
  python -m paper_2107_00820_amd.profiling rates TRACE_DIR TRAFFIC.json OUT.md --title T
      per kernel: launches and average duration from a kernel trace, HBM bytes
      per launch from the counters, and the achieved GB/s against the 8 TB/s
      HBM3E peak.
  python -m paper_2107_00820_amd.profiling mfma TRACE_DIR PMC_DIR OUT.md --title T
      per kernel: FP64 matrix-core flops per launch (SQ_INSTS_VALU_MFMA_MOPS_F64
      counts units of 512 flops) over the average duration, against the
      78.6 TFLOP/s FP64 matrix peak.

The counters are in KiB per dispatch summed over the TCC channels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


# Sources that define the star-patch GEMV kernel, its data layout and launch.
GEMV_SOURCES = ("k_patch.hip", "stk_dev.h", "stk_internal.h", "stk_ref.h")


def kernel_source_hash(files=GEMV_SOURCES) -> str:
    """Hash of the sources of the measured kernel (a change invalidates stored counters)."""
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits


def _short(name: str) -> str:
    return name.replace("void ", "").split("(")[0].strip()


def cmd_copy(args):
    import torch
    n = args.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": args.reps}))


def cmd_stats(args):
    rows = []
    for p in _find(args.dir, "*kernel_trace.csv"):
        with open(p) as f:
            rows += list(csv.DictReader(f))
    byname = collections.defaultdict(list)
    for r in rows:
        byname[_short(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    tot = sum(sum(v) for v in byname.values())
    out = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
           f"Total kernel time {tot / 1e6:.3f} ms over {len(rows)} dispatches.", "",
           "| kernel | calls | total us | avg us | share |", "|---|---:|---:|---:|---:|"]
    for k in sorted(byname, key=lambda k: -sum(byname[k]))[:30]:
        v = byname[k]
        out.append(f"| `{k}` | {len(v)} | {sum(v) / 1e3:.1f} | {sum(v) / len(v) / 1e3:.2f} | "
                   f"{100 * sum(v) / max(tot, 1):.1f}% |")
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out[:24]))


def _counter(d, counter, regex):
    """{kernel name: [KiB per dispatch]} for one counter."""
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    for p in _find(d, "*counter_collection.csv"):
        with open(p) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter or not re.search(regex, r["Kernel_Name"]):
                    continue
                acc[_short(r["Kernel_Name"])][r.get("Dispatch_Id") or r.get("Correlation_Id")] += \
                    float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def cmd_traffic(args):
    cf = _counter(args.copy_fetch, "FETCH_SIZE", args.copy_regex)
    cw = _counter(args.copy_write, "WRITE_SIZE", args.copy_regex)
    # the copy kernel: the dispatches with the largest counts
    cfv = max((v for vs in cf.values() for v in vs), default=0.0)
    cwv = max((v for vs in cw.values() for v in vs), default=0.0)
    if cfv <= 0 or cwv <= 0:
        raise SystemExit("copy kernel counters not found")
    f_fetch = args.copy_bytes / (cfv * 1024.0)
    f_write = args.copy_bytes / (cwv * 1024.0)
    kf = _counter(args.fetch, "FETCH_SIZE", args.kernel)
    kw = _counter(args.write, "WRITE_SIZE", args.kernel)
    kernels = {}
    for k in sorted(set(kf) | set(kw)):
        fv, wv = kf.get(k, []), kw.get(k, [])
        kernels[k] = {
            "launches_fetch_run": len(fv), "launches_write_run": len(wv),
            "fetch_bytes_per_launch": (sum(fv) / len(fv)) * 1024.0 * f_fetch if fv else None,
            "write_bytes_per_launch": (sum(wv) / len(wv)) * 1024.0 * f_write if wv else None,
        }
        kernels[k]["traffic_bytes_per_launch"] = (
            (kernels[k]["fetch_bytes_per_launch"] or 0.0) + (kernels[k]["write_bytes_per_launch"] or 0.0))
    out = {"command": args.cmd, "workload": args.workload, "source_hash": kernel_source_hash(),
           "copy_bytes": args.copy_bytes, "copy_fetch_kib": cfv, "copy_write_kib": cwv,
           "factor_fetch": f_fetch, "factor_write": f_write, "kernels": kernels}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


HBM_PEAK_GBS = 8000.0


def cmd_rates(args):
    rows = []
    for p in _find(args.dir, "*kernel_trace.csv"):
        with open(p) as f:
            rows += list(csv.DictReader(f))
    dur = collections.defaultdict(list)
    for r in rows:
        dur[_short(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    with open(args.traffic) as f:
        tr = json.load(f)
    c = tr.get("command", "")
    out = [f"# {args.title}", "",
           "HBM bytes per launch from `FETCH_SIZE` and `WRITE_SIZE` (two `--pmc` runs, scaled by the "
           f"copy-kernel factors {tr['factor_fetch']:.3f} / {tr['factor_write']:.3f}); average duration from "
           "the kernel trace of the same command; GB/s = bytes / duration against the 8 TB/s HBM3E peak.", "",
           "Counter commands:", "", "```", *(c if isinstance(c, list) else [c]), "```", "",
           "| kernel | launches (trace) | avg us | HBM read MB | HBM write MB | GB/s | % of peak |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    items = []
    for k, v in tr["kernels"].items():
        d = dur.get(k)
        if not d or not v.get("traffic_bytes_per_launch"):
            continue
        avg = sum(d) / len(d) / 1e3
        gbs = v["traffic_bytes_per_launch"] / (avg * 1e-6) / 1e9
        items.append((sum(d), k, len(d), avg, v, gbs))
    for _, k, n, avg, v, gbs in sorted(items, reverse=True)[:args.top]:
        out.append(f"| `{k}` | {n} | {avg:.2f} | {(v['fetch_bytes_per_launch'] or 0) / 1e6:.2f} | "
                   f"{(v['write_bytes_per_launch'] or 0) / 1e6:.2f} | {gbs:.0f} | {100 * gbs / HBM_PEAK_GBS:.1f}% |")
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


MFMA_F64_PEAK_TFLOPS = 78.6


def cmd_mfma(args):
    rows = []
    for p in _find(args.dir, "*kernel_trace.csv"):
        with open(p) as f:
            rows += list(csv.DictReader(f))
    dur = collections.defaultdict(list)
    for r in rows:
        dur[_short(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    mops = _counter(args.pmc, "SQ_INSTS_VALU_MFMA_MOPS_F64", args.kernel)
    out = [f"# {args.title}", "",
           "FP64 matrix-core flops per launch = 512 x SQ_INSTS_VALU_MFMA_MOPS_F64 (one `--pmc` run); average "
           "duration from the kernel trace of the same command; TFLOP/s against the 78.6 TFLOP/s FP64 "
           "matrix peak.", "", "Commands:", "", "```", *args.cmd, "```", "",
           "| kernel | launches (trace) | avg us | MFMA GFLOP per launch | TFLOP/s | % of peak |",
           "|---|---:|---:|---:|---:|---:|"]
    items = []
    for k, v in mops.items():
        d = dur.get(k)
        if not d or not v:
            continue
        fl = 512.0 * sum(v) / len(v)
        if fl <= 0:
            continue
        avg = sum(d) / len(d) / 1e3
        items.append((sum(d), k, len(d), avg, fl, fl / (avg * 1e-6) / 1e12))
    for _, k, n, avg, fl, tf in sorted(items, reverse=True):
        out.append(f"| `{k}` | {n} | {avg:.2f} | {fl / 1e9:.3f} | {tf:.2f} | {100 * tf / MFMA_F64_PEAK_TFLOPS:.1f}% |")
    with open(args.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("copy")
    a.add_argument("--mib", type=int, default=1024)
    a.add_argument("--reps", type=int, default=3)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--title", default="rocprofv3 kernel summary")
    a.add_argument("--cmd", default="")
    a = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out"):
        a.add_argument(k, required=True)
    a.add_argument("--copy-bytes", type=float, required=True)
    a.add_argument("--copy-regex", default="copy|elementwise|Copy")
    a.add_argument("--kernel", default="k_asm_gemv")
    a.add_argument("--workload", default="")
    a.add_argument("--cmd", default="")
    a = sub.add_parser("rates")
    a.add_argument("dir")
    a.add_argument("traffic")
    a.add_argument("out")
    a.add_argument("--title", default="achieved HBM bandwidth per kernel")
    a.add_argument("--top", type=int, default=16)
    a = sub.add_parser("mfma")
    a.add_argument("dir")
    a.add_argument("pmc")
    a.add_argument("out")
    a.add_argument("--title", default="FP64 matrix-core rate per kernel")
    a.add_argument("--kernel", default="k_patch_setup|k_sweep|k_coarse")
    a.add_argument("--cmd", action="append", default=[])
    args = ap.parse_args(argv)
    {"copy": cmd_copy, "stats": cmd_stats, "traffic": cmd_traffic, "rates": cmd_rates,
     "mfma": cmd_mfma}[args.cmd_name](args)


if __name__ == "__main__":
    sys.exit(main())
