"""Summaries of rocprofv3 output for the kernels of libaao.

    python -m paper_1810_00615_amd.profiling trace DIR [--cmd "..."]
        per-kernel-family duration table (markdown) from DIR/*_kernel_trace.csv

    python -m paper_1810_00615_amd.profiling traffic FETCH_DIR WRITE_DIR --family matvec
            --alg-bytes B --copy-bytes C --source FILE... [--cmd "..."]
        HBM bytes per launch of one kernel family from a FETCH_SIZE run and a
        WRITE_SIZE run (KiB per dispatch), each scaled by the ratio of the known
        bytes of a plain device copy of C bytes (read C, write C; the largest copy
        dispatch of the run) to what the same counter reads for that copy; prints a
        JSON record keyed by the sha256 of the kernel sources.

Kernel families group template instantiations: "k_matvec<1, 8, true, false>" and
"k_matvec<1, 8, true, true>" both belong to "matvec".
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

FAMILIES = [
    ("fft_fwd", r"k_fft_fwd|k_dft_fwd|k_batch_fft_fwd"),
    ("fft_inv", r"k_fft_inv|k_dft_inv|k_batch_fft_inv"),
    ("shifted_solve", r"k_shifted_solve|k_batch_solve"),
    ("matvec", r"k_matvec|k_batch_matvec"),
    ("cgs", r"k_cgs|k_batch_cgs"),
    ("reduce", r"k_reduce_small|k_reduce_parts|k_batch_reduce|k_batch_small"),
    ("axpy", r"k_multi_axpy|k_batch_axpy"),
    ("arnoldi_update", r"k_arnoldi_update"),
    ("sine_y", r"k_dst_y"),
    ("dot", r"k_dot1"),
    ("copy", r"copyBuffer|elementwise_kernel.*copy|direct_copy"),
]


def family(name: str) -> str:
    for fam, pat in FAMILIES:
        if re.search(pat, name):
            return fam
    return "other"


def short(name: str) -> str:
    return re.sub(r"\(.*", "", name).replace("aao::", "").replace("void ", "")


def _rows(d, suffix):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    out = []
    for f in files:
        out.extend(csv.DictReader(open(f)))
    return out


def trace_table(d, cmd=None):
    rows = _rows(d, "_kernel_trace.csv")
    per = {}
    for r in rows:
        k = short(r["Kernel_Name"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per.setdefault(k, []).append(dur)
    lines = []
    if cmd:
        lines += [f"Command: `{cmd}`", ""]
    lines += ["| kernel | family | calls | avg us | median us | total us |",
              "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        v2 = sorted(v)
        lines.append(f"| `{k}` | {family(k)} | {len(v)} | {sum(v) / len(v):.1f} | "
                     f"{v2[len(v2) // 2]:.1f} | {sum(v):.1f} |")
    fams = {}
    for k, v in per.items():
        f = family(k)
        a = fams.setdefault(f, [0, 0.0])
        a[0] += len(v)
        a[1] += sum(v)
    lines += ["", "| family | calls | avg us | total us |", "|---|---|---|---|"]
    for f, (c, t) in sorted(fams.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {f} | {c} | {t / c:.1f} | {t:.1f} |")
    stats = glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True)
    if stats:
        lines += ["", "rocprofv3 --stats summary (`*_kernel_stats.csv`):", "",
                  "| kernel | calls | avg us | min us | max us | percent |",
                  "|---|---|---|---|---|---|"]
        for f in stats:
            for r in csv.DictReader(open(f)):
                lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | "
                             f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                             f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def _counter(d, counter):
    rows = _rows(d, "_counter_collection.csv")
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def traffic_record(fetch_dir, write_dir, fam, alg_bytes, copy_bytes, sources, cmd=None,
                   kernel_filter=None):
    fetch = _counter(fetch_dir, "FETCH_SIZE")
    write = _counter(write_dir, "WRITE_SIZE")

    def pick(tab, want):
        vals = []
        for k, v in tab.items():
            if family(k) == want and (kernel_filter is None or re.search(kernel_filter, k)
                                      or want == "copy"):
                vals.extend(v)
        if not vals:
            raise SystemExit(f"no {want} dispatches in the counter output")
        return sum(vals) / len(vals), len(vals)

    def largest_copy(tab):
        vals = [x for k, v in tab.items() if family(k) == "copy" for x in v]
        if not vals:
            raise SystemExit("no copy dispatch in the counter output (run with a calibration copy)")
        return max(vals)

    cf = largest_copy(fetch)   # the calibration copy is the largest copy dispatch
    cw = largest_copy(write)
    kf, nf = pick(fetch, fam)
    kw, nw = pick(write, fam)
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    h = hashlib.sha256()
    for s in sources:
        h.update(open(s, "rb").read())
    rec = {
        "kernel": fam,
        "bytes_per_launch": kf * 1024.0 * f_scale + kw * 1024.0 * w_scale,
        "fetch_KiB_per_dispatch": kf, "write_KiB_per_dispatch": kw,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "dispatches": [nf, nw],
        "alg_bytes_per_launch": alg_bytes,
        "traffic_over_alg": (kf * 1024.0 * f_scale + kw * 1024.0 * w_scale) / alg_bytes
        if alg_bytes else None,
        "sources": sources,
        "source_sha256_16": h.hexdigest()[:16],
    }
    if cmd:
        rec["command"] = cmd
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--cmd")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("--family", required=True)
    f.add_argument("--kernel-filter")
    f.add_argument("--alg-bytes", type=float, default=None)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--source", nargs="+", required=True)
    f.add_argument("--cmd")
    a = ap.parse_args(argv)
    if a.what == "trace":
        print(trace_table(a.dir, a.cmd))
    else:
        print(json.dumps(traffic_record(a.fetch_dir, a.write_dir, a.family, a.alg_bytes,
                                        a.copy_bytes, a.source, a.cmd, a.kernel_filter),
                         indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
