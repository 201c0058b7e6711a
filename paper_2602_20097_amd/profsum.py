"""Summaries of rocprofv3 runs of bench.py (kernel time and HBM traffic).

    python -m paper_2602_20097_amd.profsum --trace DIR [--fetch DIR --write DIR]
           --workload NAME --out profiles/NAME.md [--commands FILE]

DIR holds the CSV output of one rocprofv3 run (``--output-format csv``):
``*_kernel_stats.csv`` for ``--kernel-trace --stats``, ``*_counter_collection.csv``
for a ``--pmc`` run.  FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch and
scaled by what the same counters report for the copy probe (``k_copy``), whose
bytes are known: n words read and n words written.  The per-stage bytes per
launch go to ``profiles/traffic.json`` under ``workload:stage`` together with a
hash of the kernel sources, so that bench.py only reports them while the
kernels are the ones that were measured.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# kernel symbol -> bench stage (the plain path launches one kernel per stage)
STAGES = [
    (r"k_seed_(lane|seg|slab|xscan|lines)<0", "seed1_xscan"),
    (r"k_seed_(lane|seg|slab|xscan|lines)<1", "seed2_xscan"),
    (r"k_interp_own", "edt2_z_interp"),
    (r"k_interp_pre", "edt2_z_stream"),
    (r"k_interp_far", "edt2_z_search"),
    (r"k_interp_dir", "edt2_y_interp"),
    (r"k_env_lane2_z", "edt2_z_sparse"),
    (r"k_edt1_yz", "edt1_yz"),
    (r"k_env_lane2_y\b", "edt2_y"),
    (r"k_interp\b", "interp"),
    (r"k_copy", "copy_probe"),
    (r"k_clear", "clear"),
]
SEED1 = r"k_seed_(lane|seg|slab|xscan|lines)<0"
SEED2 = r"k_seed_(lane|seg|slab|xscan|lines)<1"


# the sources of the plain pass's kernels (the ones the traffic figures cover)
REV_SOURCES = ("qai_plain.hip", "qai_device.h", "qai_code.h")


def kernel_rev():
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2602_20097_amd", "csrc")
    for f in REV_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def _one(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[-1]


def stage_of(name, order, fused=False):
    """Envelope passes are told apart by their order within a step: the first
    EDT's y and z passes come before the second seed pass; after the fused
    y/z search of the first EDT they are its gated fallback."""
    for pat, st in STAGES:
        if re.search(pat, name):
            return st
    if re.search(r"k_env_\w+<[12]", name) and order == 0 and fused:
        return "edt1_fallback"
    if re.search(r"k_env_\w+<1", name):
        return "edt1_y" if order == 0 else "edt2_y"
    if re.search(r"k_env_\w+<2", name):
        return "edt1_z" if order == 0 else "edt2_z"
    return None


def read_stats(d):
    rows = []
    with open(_one(os.path.join(d, "**", "*kernel_stats.csv"))) as fh:
        for r in csv.DictReader(fh):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]), "total_ns": float(r["TotalDurationNs"]),
                         "avg_ns": float(r["AverageNs"]), "pct": float(r["Percentage"])})
    return rows


def _per_step(events):
    """events: (name, value) in dispatch order.  A step starts at its first
    seed kernel; the values of a stage's kernels are summed within a step and
    averaged over steps (the copy probe, outside the steps, per launch)."""
    steps, cur, seen_seed2, fused = [], None, False, False
    copy = []
    for name, val in events:
        if re.search(SEED1, name):
            cur = {}
            steps.append(cur)
            seen_seed2 = fused = False
        if re.search(SEED2, name):
            seen_seed2 = True
        if re.search(r"k_edt1_yz", name):
            fused = True
        st = stage_of(name, 1 if seen_seed2 else 0, fused)
        if st == "copy_probe":
            copy.append(val)
        elif st and cur is not None:
            cur[st] = cur.get(st, 0.0) + val
    out = {}
    for st in sorted({k for s in steps for k in s}):
        vals = [s[st] for s in steps if st in s]
        out[st] = (statistics.mean(vals), len(vals))
    if copy:
        out["copy_probe"] = (statistics.mean(copy), len(copy))
    return out


def read_trace_stages(d):
    """Per-stage duration per step from the kernel trace (dispatch order decides
    which envelope kernel belongs to which EDT)."""
    path = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    with open(path) as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    return _per_step([(r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows])


def read_counter(d, counter):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    disp = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            name, val = r["Kernel_Name"], float(r["Counter_Value"])
            disp.setdefault(key, [name, 0.0])[1] += val
    per = _per_step([tuple(disp[k]) for k in sorted(disp)])
    return {k: v[0] for k, v in per.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--voxels", type=int, required=True)
    ap.add_argument("--copy-words", type=int, required=True, help="words the copy probe moves per launch")
    ap.add_argument("--out", required=True)
    ap.add_argument("--commands", required=True, help="text file with the exact profiling commands")
    args = ap.parse_args()

    stats = read_stats(args.trace)
    stages = read_trace_stages(args.trace)
    lines = [f"# rocprofv3 summary: {args.workload} ({args.voxels} voxels), plain path", "",
             "Commands (run from the repository root on one MI355X):", "", "```"]
    lines += open(args.commands).read().strip().splitlines()
    lines += ["```", "", "## Kernel statistics (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -r["total_ns"]):
        nm = r["name"].replace("|", "/")
        lines.append(f"| `{nm[:90]}` | {r['calls']} | {r['avg_ns'] / 1e3:.1f} | {r['total_ns'] / 1e6:.2f} | "
                     f"{r['pct']:.1f} |")
    lines += ["", "## Per stage and step (kernel trace, dispatch order; a stage's kernels summed)", "",
              "| stage | steps | avg us |", "|---|---|---|"]
    for st, (avg, cnt) in stages.items():
        lines.append(f"| {st} | {cnt} | {avg / 1e3:.1f} |")

    if args.fetch and args.write:
        fetch = read_counter(args.fetch, "FETCH_SIZE")
        write = read_counter(args.write, "WRITE_SIZE")
        copy_bytes = 4.0 * args.copy_words
        kf = copy_bytes / (fetch["copy_probe"] * 1024.0)
        kw = copy_bytes / (write["copy_probe"] * 1024.0)
        lines += ["", "## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE)", "",
                  f"Scale factors from the copy probe ({args.copy_words} words each way): "
                  f"fetch x{kf:.3f}, write x{kw:.3f}.", "",
                  "| stage | fetch MiB (raw) | write MiB (raw) | bytes/step (scaled) | bytes/voxel |",
                  "|---|---|---|---|---|"]
        tfile = os.path.join(ROOT, "profiles", "traffic.json")
        tr = {}
        if os.path.exists(tfile):
            with open(tfile) as fh:
                tr = json.load(fh)
        rev = kernel_rev()
        for st in fetch:
            if st not in write or st == "copy_probe":
                continue
            b = fetch[st] * 1024.0 * kf + write[st] * 1024.0 * kw
            lines.append(f"| {st} | {fetch[st] / 1024:.1f} | {write[st] / 1024:.1f} | {b:.4g} | "
                         f"{b / args.voxels:.2f} |")
            tr[f"{args.workload}:{st}"] = {"bytes_per_launch": round(b), "kernel_rev": rev}
        with open(tfile, "w") as fh:
            json.dump(tr, fh, indent=1, sort_keys=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
