"""Summaries of rocprofv3 output for the benchmark's kernels.

* ``stats``: the kernel statistics CSV of ``rocprofv3 --kernel-trace --stats
  --output-format csv`` turned into a short Markdown table (calls, mean and
  total duration per kernel).
* ``traffic``: two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` counter runs of
  a command, plus the same two runs of a device-to-device copy of known size,
  turned into HBM bytes per launch of the named kernels.  The counters read in
  KiB; each is scaled by the factor (bytes the copy must move) / (bytes the
  counter reports for it), so a kernel's figure is in the copy's units.

    python -m paper_2412_18379_amd.profiling stats <kernel_stats.csv> <out.md> "<command>" [+names|-names]
    python -m paper_2412_18379_amd.profiling traffic <fetch.csv> <write.csv> <copy_fetch.csv> \
        <copy_write.csv> <copy_bytes> <workload> <traffic.json> "<command>" name=kernel[*k][+kernel[*k]] ...

  (a kernel is named by substrings of its full name joined with "&"; "*k"
  counts it k times per launch of the group)
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# the source file(s) each benchmark kernel group is built from
SOURCES = {
    "cnn_forward_f32": ("cnn.hip",),
    "cnn_forward_bf16": ("cnn_bf16.hip",),
    "k_locate_plain": ("sns_walk.hip",),
    "k_locate_cnn": ("sns_walk.hip",),
    "k_interp": ("sns_walk.hip",),
    "k3_locate_plain": ("mesh3d.hip",),
    "k3_locate_lookup": ("mesh3d.hip",),
    "k3_locate_cnn": ("mesh3d.hip",),
    "k3_interp": ("mesh3d.hip",),
    "cnn3_forward_f32": ("cnn3d.hip",),
    "cnn3_forward_bf16": ("cnn3d.hip",),
}


def source_sha(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(HERE, "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str, width: int = 90) -> str:
    """Kernel name without its argument list (and cut to width characters)."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        out.append(ch)
    short = "".join(out).strip()
    return short if len(short) <= width else short[:width - 3] + "..."


def stats(csv_path: str, out_path: str, command: str, top: int = 20, select: str = "") -> str:
    """Markdown table of the kernel statistics; `select` "+a,b" keeps only the kernels whose name
    contains one of a, b, "-a,b" drops them (the percentages stay those of the whole run)."""
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    if select:
        keys = select[1:].split(",")
        keep = select[0] == "+"
        rows = [r for r in rows if any(k in r["Name"] for k in keys) == keep]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"Command: `{command}`", "",
             "| kernel | calls | mean (us) | min (us) | max (us) | total (ms) | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as f:
        f.write(text)
    return text


def _per_kernel(csv_path: str, counter: str):
    """Mean counter value (KiB) per dispatch, by kernel name."""
    tot, cnt = defaultdict(float), defaultdict(int)
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            tot[r["Kernel_Name"]] += float(r["Counter_Value"])
            cnt[r["Kernel_Name"]] += 1
    return {k: (tot[k] / cnt[k], cnt[k]) for k in tot}


def _match(table, substrings):
    hits = [(k, v) for k, v in table.items() if all(s in k for s in substrings)]
    if not hits:
        raise KeyError(f"no kernel matches {substrings}")
    if len(hits) > 1:
        hits.sort(key=lambda kv: -kv[1][1])
    return hits[0]


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, workload, out_json, command, groups):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    cf = _per_kernel(copy_fetch_csv, "FETCH_SIZE")
    cw = _per_kernel(copy_write_csv, "WRITE_SIZE")
    copy_name = max(cf, key=lambda k: cf[k][0])
    f_scale = copy_bytes / (cf[copy_name][0] * 1024.0)
    w_scale = copy_bytes / (cw[copy_name][0] * 1024.0)
    db = {}
    if os.path.exists(out_json):
        with open(out_json) as f:
            db = json.load(f)
    for name, subs in groups.items():
        total_r = total_w = 0.0
        kernels = []
        for sub in subs:
            sub, _, times = sub.partition("*")  # "name*k": the kernel runs k times per launch of the group
            times = int(times or 1)
            kf, (vf, nf) = _match(fetch, sub.split("&"))
            kw, (vw, nw) = _match(write, sub.split("&"))
            total_r += times * vf * 1024.0 * f_scale
            total_w += times * vw * 1024.0 * w_scale
            kernels.append({"kernel": _short(kf), "per_group_launch": times, "fetch_KiB": round(vf, 1),
                            "write_KiB": round(vw, 1), "dispatches": nf})
        db[f"{name}@{workload}"] = {
            "hbm_bytes_per_launch": round(total_r + total_w),
            "read_bytes": round(total_r), "write_bytes": round(total_w),
            "kernels": kernels, "source_sha": source_sha(*SOURCES[name]),
            "copy_calibration": {"kernel": _short(copy_name), "bytes": copy_bytes,
                                 "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
            "command": command,
        }
    with open(out_json, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    return db


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4], select=sys.argv[5] if len(sys.argv) > 5 else ""))
    elif sys.argv[1] == "traffic":
        a = sys.argv[2:]
        groups = {}
        for g in a[8:]:
            k, v = g.split("=", 1)
            groups[k] = v.split("+")
        print(json.dumps(traffic(a[0], a[1], a[2], a[3], int(a[4]), a[5], a[6], a[7], groups), indent=1))
    else:
        raise SystemExit(__doc__)
