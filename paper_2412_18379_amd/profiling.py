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
        <copy_write.csv> <copy_bytes> <workload> <traffic.json> "<command>" name=kernel[*k][+kernel[*k]] ... \
        [rdreq=<rdreq.csv> copy_rdreq=<copy_rdreq.csv>]
    python -m paper_2412_18379_amd.profiling counters <out.md> <kernel_stats.csv> "<commands>" \
        <counter_collection.csv> [more counter csvs] -- substring[,substring ...]

* ``counters``: per kernel (name containing one of the substrings), the mean
  per dispatch of every counter in the given --pmc runs, the mean duration
  from a --kernel-trace --stats run, and what follows from them: the
  matrix-core busy fraction (MfmaUtil), the matrix FLOPs per dispatch
  (MfmaFlopsF32 / MfmaFlopsBF16, 512 per MOP) and their rate against the
  duration, and HBM-side read bytes from the TCC/EA read requests counted
  by size (TCC_EA0_RDREQ_32B / _64B / _128B), with the share sent to DRAM.

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
    "cnn_forward_f32": ("cnn.hip", "strip.h"),
    "cnn_forward_bf16": ("cnn_bf16.hip",),
    "cnn_forward_fp8": ("cnn_fp8.hip",),
    "k_locate_plain": ("sns_walk.hip",),
    "k_locate_cnn": ("sns_walk.hip",),
    "k_interp": ("sns_walk.hip",),
    "k_locate_cnn_interp": ("sns_walk.hip",),
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


def _request_bytes(csv_path):
    """{kernel: (HBM-side read bytes per dispatch from the TCC read requests counted by size, dispatches)}."""
    table = _counter_table([csv_path])
    out = {}
    for k, c in table.items():
        if "TCC_EA0_RDREQ_64B_sum" not in c:
            continue
        out[k] = (32 * c.get("TCC_EA0_RDREQ_32B_sum", 0.0) + 64 * c["TCC_EA0_RDREQ_64B_sum"] +
                  128 * c.get("TCC_EA0_RDREQ_128B_sum", 0.0), 1)
    return out


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, workload, out_json, command, groups,
            rdreq_csv=None, copy_rdreq_csv=None):
    """HBM bytes per launch of each kernel group.  With rdreq_csv (a --pmc run of TCC_EA0_RDREQ_32B/_64B/
    _128B_sum) the read side is also given from the requests counted by size, unscaled, beside the
    copy-scaled FETCH_SIZE figure: the copy moves 128-byte lines, a gather of 64-byte records does not,
    so one scale factor cannot serve both."""
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    cf = _per_kernel(copy_fetch_csv, "FETCH_SIZE")
    cw = _per_kernel(copy_write_csv, "WRITE_SIZE")
    copy_name = max(cf, key=lambda k: cf[k][0])
    f_scale = copy_bytes / (cf[copy_name][0] * 1024.0)
    w_scale = copy_bytes / (cw[copy_name][0] * 1024.0)
    req = _request_bytes(rdreq_csv) if rdreq_csv else None
    copy_req = _request_bytes(copy_rdreq_csv) if copy_rdreq_csv else None
    db = {}
    if os.path.exists(out_json):
        with open(out_json) as f:
            db = json.load(f)
    for name, subs in groups.items():
        total_r = total_w = total_q = 0.0
        kernels = []
        for sub in subs:
            sub, _, times = sub.partition("*")  # "name*k": the kernel runs k times per launch of the group
            times = int(times or 1)
            kf, (vf, nf) = _match(fetch, sub.split("&"))
            kw, (vw, nw) = _match(write, sub.split("&"))
            total_r += times * vf * 1024.0 * f_scale
            total_w += times * vw * 1024.0 * w_scale
            entry = {"kernel": _short(kf), "per_group_launch": times, "fetch_KiB": round(vf, 1),
                     "write_KiB": round(vw, 1), "dispatches": nf}
            if req is not None:
                kq, (vq, _) = _match(req, sub.split("&"))
                total_q += times * vq
                entry["read_bytes_by_request_size"] = round(vq)
            kernels.append(entry)
        rec = db[f"{name}@{workload}"] = {
            "hbm_bytes_per_launch": round(total_r + total_w),
            "read_bytes": round(total_r), "write_bytes": round(total_w),
            "kernels": kernels, "source_sha": source_sha(*SOURCES[name]),
            "copy_calibration": {"kernel": _short(copy_name), "bytes": copy_bytes,
                                 "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
            "command": command,
        }
        if req is not None:
            rec["read_bytes_by_request_size"] = round(total_q)
            rec["hbm_bytes_per_launch_by_request_size"] = round(total_q + total_w)
            if copy_req:
                cq = max(copy_req.values(), key=lambda v: v[0])[0]
                rec["copy_calibration"]["read_bytes_by_request_size"] = round(cq)
    with open(out_json, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    return db


def _counter_table(csv_paths):
    """{kernel: {counter: mean per dispatch}} over one or more --pmc CSVs."""
    tot, cnt = defaultdict(lambda: defaultdict(float)), defaultdict(lambda: defaultdict(int))
    for path in csv_paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                k, c = r["Kernel_Name"], r["Counter_Name"]
                tot[k][c] += float(r["Counter_Value"])
                cnt[k][c] += 1
    return {k: {c: tot[k][c] / cnt[k][c] for c in tot[k]} for k in tot}


def counters(out_path, stats_csv, command, csv_paths, select):
    table = _counter_table(csv_paths)
    durations = {}
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            durations[r["Name"]] = float(r["AverageNs"])
    keys = select.split(",")
    names = sorted((k for k in table if any(s in k for s in keys)), key=lambda k: _short(k))
    lines = [f"Commands: `{command}`", "",
             "| kernel | mean (us) | MFMA busy | MFMA TFLOP/dispatch (F32 / BF16) | MFMA TFLOP/s | "
             "VALU instr / dispatch | HBM-side read bytes / dispatch | to DRAM |",
             "|---|---|---|---|---|---|---|---|"]
    out = {}
    for k in names:
        c = table[k]
        dur = durations.get(k)
        f32, b16 = c.get("MfmaFlopsF32"), c.get("MfmaFlopsBF16")
        flops = (f32 or 0.0) + (b16 or 0.0)
        rate = flops / (dur * 1e-9) / 1e12 if dur and flops else None
        rd = None
        if "TCC_EA0_RDREQ_128B_sum" in c and "TCC_EA0_RDREQ_64B_sum" in c:
            rd = (128 * c["TCC_EA0_RDREQ_128B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"] +
                  32 * c.get("TCC_EA0_RDREQ_32B_sum", 0.0))
        dram = (c["TCC_EA0_RDREQ_DRAM_sum"] / c["TCC_EA0_RDREQ_sum"]
                if c.get("TCC_EA0_RDREQ_sum") and "TCC_EA0_RDREQ_DRAM_sum" in c else None)
        row = {"mean_us": dur / 1e3 if dur else None, "mfma_util": c.get("MfmaUtil"),
               "mfma_flops_f32": f32, "mfma_flops_bf16": b16, "mfma_tflops": rate,
               "valu_insts": c.get("SQ_INSTS_VALU"), "read_bytes": rd, "dram_share": dram,
               "counters": {n: round(v, 3) for n, v in sorted(c.items())}}
        out[_short(k)] = row

        def fmt(v, spec):
            return "—" if v is None else format(v, spec)
        lines.append(f"| `{_short(k)}` | {fmt(row['mean_us'], '.1f')} | "
                     f"{fmt(row['mfma_util'] and row['mfma_util'] / 100, '.3f')} | "
                     f"{fmt(f32 and f32 / 1e12, '.4f')} / {fmt(b16 and b16 / 1e12, '.4f')} | {fmt(rate, '.1f')} | "
                     f"{fmt(row['valu_insts'], '.4g')} | {fmt(rd, '.4g')} | {fmt(dram, '.3f')} |")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as f:
        f.write(text)
    with open(os.path.splitext(out_path)[0] + ".json", "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    return text


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4], select=sys.argv[5] if len(sys.argv) > 5 else ""))
    elif sys.argv[1] == "traffic":
        a = sys.argv[2:]
        groups, extra = {}, {}
        for g in a[8:]:
            k, v = g.split("=", 1)
            if k in ("rdreq", "copy_rdreq"):
                extra[k + "_csv"] = v
            else:
                groups[k] = v.split("+")
        print(json.dumps(traffic(a[0], a[1], a[2], a[3], int(a[4]), a[5], a[6], a[7], groups, **extra), indent=1))
    elif sys.argv[1] == "counters":
        a = sys.argv[2:]
        sep = a.index("--")
        print(counters(a[0], a[1], a[2], a[3:sep], a[sep + 1]))
    else:
        raise SystemExit(__doc__)
