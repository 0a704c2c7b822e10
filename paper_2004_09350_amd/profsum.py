"""Summaries of rocprofv3 output for profiles/ (kernel statistics and HBM traffic).

    python -m paper_2004_09350_amd.profsum <trace_dir> <fetch_dir> <write_dir> <out_prefix> [--traffic=NAME] <command...>

reads <trace_dir>/*_kernel_stats.csv (``rocprofv3 --kernel-trace --stats``), the
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` counter collections and the fetch run's log
(<fetch_dir>.log), and writes <out_prefix>.md (top kernels by time, average durations,
per-dispatch traffic) and profiles/NAME.json (default ``traffic``; per kernel: HBM bytes
per launch, the figure bench.py reports for the same workload: ``traffic`` for the
sweep, ``traffic_star`` etc. for the plan workloads).

Counter scaling: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by
known / measured for the reference copy kernel ``k_decode`` of an uncompressed column
(4 bytes read and 4 bytes written per row), launched once by ``bench.py --calib-copy``.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short(name: str) -> str:
    n = re.sub(r"\(.*\)$", "", name)
    n = n.replace("void ", "").replace("ms::", "").replace("(anonymous namespace)::", "")
    n = re.sub(r"<(\d+)u>", r"<\1>", n)
    return n


KIND_NAMES = ("UNCOMPR", "STATIC_BP", "DYN_BP", "DELTA_DYN_BP", "FOR_DYN_BP", "RLE")


def canonical(name: str) -> str:
    """Kernel names as the library's launch timer reports them (k_morph<DYN_BP>, k_pred<0>)."""
    n = short(name)
    m = re.match(r"(k_morph|k_project|k_project_rle)<(\d+)>", n)
    if m:
        return f"{m.group(1)}<{KIND_NAMES[int(m.group(2))]}>"
    return n


def counters(d: str, counter: str):
    f = glob.glob(os.path.join(d, "*_counter_collection.csv"))[0]
    per = defaultdict(list)
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] == counter:
            per[canonical(r["Kernel_Name"])].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return per


def main(argv):
    trace_dir, fetch_dir, write_dir, out_prefix = argv[:4]
    rest = argv[4:]
    traffic_name = "traffic"  # profiles/<name>.json, read by bench.py for the same workload
    if rest and rest[0].startswith("--traffic="):
        traffic_name = rest[0].split("=", 1)[1]
        rest = rest[1:]
    command = " ".join(rest)
    stats = list(csv.DictReader(open(glob.glob(os.path.join(trace_dir, "*_kernel_stats.csv"))[0])))
    fetch = counters(fetch_dir, "FETCH_SIZE")
    write = counters(write_dir, "WRITE_SIZE")
    # calibration: the first k_decode dispatch is the reference copy (bench --calib-copy)
    rows = None
    for line in open(fetch_dir.rstrip("/") + ".log"):
        m = re.search(r"calibration copy: k_decode of (\d+) rows", line)
        if m:
            rows = int(m.group(1))
    if rows is None or "k_decode" not in fetch or "k_decode" not in write:
        raise SystemExit("calibration dispatch missing")
    known = 4.0 * rows
    f_fetch = known / (fetch["k_decode"][0][1] * 1024)
    f_write = known / (write["k_decode"][0][1] * 1024)
    sys.path.insert(0, ROOT)
    from bench import source_sha
    traffic = {"source_sha": source_sha(), "fetch_scale": f_fetch, "write_scale": f_write,
               "command": command, "kernels": {}}
    for k in sorted(set(fetch) & set(write)):
        fv = [v for _, v in fetch[k]]
        wv = [v for _, v in write[k]]
        traffic["kernels"][k] = {
            "dispatches": len(fv),
            "fetch_bytes_per_launch": sum(fv) / len(fv) * 1024 * f_fetch,
            "write_bytes_per_launch": sum(wv) / len(wv) * 1024 * f_write,
            "bytes_per_launch": (sum(fv) / len(fv) * 1024 * f_fetch + sum(wv) / len(wv) * 1024 * f_write),
        }
    json.dump(traffic, open(os.path.join(ROOT, "profiles", traffic_name + ".json"), "w"), indent=1)
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    lines = [f"# rocprofv3 kernel statistics: {os.path.basename(out_prefix)}", "",
             f"Command (from the repository root): `rocprofv3 --kernel-trace --stats -d <dir> -o trace "
             f"--output-format csv -- {command}`", "",
             f"HBM traffic: two more runs of the same command with `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE`; "
             f"counters scaled by the reference copy (k_decode of {rows} uncompressed rows): "
             f"fetch x{f_fetch:.4f}, write x{f_write:.4f}.  Summarised with "
             f"`python -m paper_2004_09350_amd.profsum <trace_dir> <fetch_dir> <write_dir> <out_prefix> <command>`.",
             "", f"Source hash of the kernels profiled: {traffic['source_sha']}", "",
             "| kernel | calls | total ms | avg us | % time | HBM read MB/launch | HBM write MB/launch |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        k = canonical(r["Name"])
        t = traffic["kernels"].get(k)
        rd = f"{t['fetch_bytes_per_launch'] / 1e6:.2f}" if t else "-"
        wr = f"{t['write_bytes_per_launch'] / 1e6:.2f}" if t else "-"
        lines.append(f"| {k} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / total:.1f} | "
                     f"{rd} | {wr} |")
    open(out_prefix + ".md", "w").write("\n".join(lines) + "\n")
    print(out_prefix + ".md")


if __name__ == "__main__":
    main(sys.argv[1:])
