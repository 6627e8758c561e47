"""Summaries of rocprofv3 output for the decoder kernels.

    python -m paper_2607_27644_amd.profiling stats  <kernel_stats.csv> <out.md> [title] [command]
    python -m paper_2607_27644_amd.profiling traffic <fetch_counter.csv> <write_counter.csv> <kernel substring>
                                                   <copy MiB> <shots> <workload> <out.json>

`traffic` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the named kernel
by the ratio of known bytes to counted bytes of the calibration copy kernel in
the same run, and records the hash of the kernel sources it was taken on.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("rbp_decode.hip", "rbp_common.h"):
        h.update(open(os.path.join(ROOT, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stats_md(path: str, out: str, title: str = "", command: str = ""):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# {title or 'rocprofv3 kernel statistics'}", ""]
    if command:
        lines += ["Command:", "", "```", command, "```", ""]
    lines += ["| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter (summed over dimensions)."""
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        acc[r["Dispatch_Id"]] += float(r["Counter_Value"])
        names[r["Dispatch_Id"]] = r["Kernel_Name"]
    out = defaultdict(list)
    for d, v in sorted(acc.items(), key=lambda kv: int(kv[0])):
        out[names[d]].append(v)
    return out


def traffic(fetch_csv, write_csv, kernel_sub, copy_mib, shots, workload, out):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    copy_bytes = float(copy_mib) * (1 << 20)

    def pick(d, sub):
        for k, v in d.items():
            if sub in k:
                return k, v
        raise KeyError(sub)

    _, cf = pick(fetch, "copy")
    _, cw = pick(write, "copy")
    f_scale = copy_bytes / (max(cf) * 1024.0)
    w_scale = copy_bytes / (max(cw) * 1024.0)
    kname, kf = pick(fetch, kernel_sub)
    _, kw = pick(write, kernel_sub)
    fb = kf[-1] * 1024.0 * f_scale
    wb = kw[-1] * 1024.0 * w_scale
    rec = {"kernel": kname, "workload": workload, "shots": int(shots), "kernel_source_hash": kernel_source_hash(),
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb,
           "calibration": {"copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
                           "copy_fetch_kib": max(cf), "copy_write_kib": max(cw)},
           "raw_kib": {"fetch": kf, "write": kw}}
    json.dump(rec, open(out, "w"), indent=1)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_md(sys.argv[2], sys.argv[3], *(sys.argv[4:6]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:9]), indent=1))
    else:
        raise SystemExit(__doc__)
