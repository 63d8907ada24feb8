"""Summaries of rocprofv3 output for the profiles folder.

    python rocprof_summary.py stats DIR OUT.md --cmd "..." [--note "..."]
        kernel statistics (``--kernel-trace --stats --output-format csv``) as a
        markdown table, with the command that produced them.
    python rocprof_summary.py counters DIR OUT.md --kernels k_a k_b --cmd "..." [--note "..."]
        median per dispatch of each SQ / GRBM counter of one ``--pmc`` run for
        the named kernels, with the derived matrix-core ratios.
    python rocprof_summary.py traffic --workload W --fetch DIR --write DIR \\
            --copy-fetch DIR --copy-write DIR --copy-bytes B --kernels k_forward k_adjoint --out OUT.md
        HBM traffic per launch from two counter runs (FETCH_SIZE, then
        WRITE_SIZE, KiB per dispatch), each scaled by the same counter's
        reading for a plain device-to-device copy of B bytes; the result is
        merged into profiles/traffic.json under W with the hash of the DFT
        kernel source (the benchmark reports it only while the hash matches).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


def _demangle(name: str) -> str:
    """Readable form of this library's mangled kernel names (the system
    demangler does not know the 16-bit float types): function name and
    template arguments."""
    m = re.match(r"_ZN(?:\d+\w+?)*?12_GLOBAL__N_1(\d+)", name)
    if not m:
        return name
    start = m.end()
    fn = name[start:start + int(m.group(1))]
    rest = name[start + int(m.group(1)):]
    args = []
    if rest.startswith("I"):
        rest = rest[1:]
        tok = {"DF16b": "__bf16", "DF16_": "_Float16", "f": "float", "d": "double"}
        while rest and not rest.startswith("E"):
            t = re.match(r"Li(\d+)E", rest)
            if t:
                args.append(t.group(1))
                rest = rest[t.end():]
                continue
            for k, v in tok.items():
                if rest.startswith(k):
                    args.append(v)
                    rest = rest[len(k):]
                    break
            else:
                break
    return f"uvm::{fn}<{', '.join(args)}>" if args else f"uvm::{fn}"


def _short(name: str) -> str:
    s = _demangle(name).replace("(anonymous namespace)::", "")
    s = re.sub(r"\(.*", "", s)
    return s.strip()


def _one(dirpath: str, pattern: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirpath, "**", pattern), recursive=True))
    if not hits:
        sys.exit(f"no {pattern} under {dirpath}")
    return hits[0]


def stats(args):
    path = _one(args.dir, "*kernel_stats.csv")
    with open(path) as f:
        rows = list(csv.DictReader(f))
    lines = [f"# {args.title}", "", "Command (repository root, one MI355X):", "", "```",
             "cd /tmp && export TMPDIR=/tmp && cd -", args.cmd, "```", ""]
    if args.note:
        lines += [args.note, ""]
    lines += [f"Source: `{os.path.basename(path)}`.", "",
              "| kernel | calls | total ms | avg us | min us | max us | % |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{_short(r['Name'])[:70]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}")


def _counter(dirpath: str, counter: str):
    """{short kernel name: [values per dispatch]} for one counter."""
    path = _one(dirpath, "*counter_collection.csv")
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def _fname(name: str) -> str:
    """Function name of a kernel name, demangled (uvm::k_adjoint_h16<...>) or
    mangled (_ZN3uvm12_GLOBAL__N_113k_adjoint_h16I...): k_adjoint_h16."""
    m = re.match(r"_ZN(?:\d+\w+?)*?12_GLOBAL__N_1(\d+)", name)
    if m:
        start = m.end()
        return name[start:start + int(m.group(1))]
    m = re.search(r"(\w+)\s*(<|$)", name)
    return m.group(1) if m else name


def _match(d, key):
    vals = [v for k, vs in d.items() if _fname(k) == key for v in vs]
    if not vals:
        sys.exit(f"no dispatch of {key}")
    return statistics.median(vals), len(vals)


def traffic(args):
    sys.path.insert(0, ROOT)
    from bench import kernel_hash

    f_k, w_k = _counter(args.fetch, "FETCH_SIZE"), _counter(args.write, "WRITE_SIZE")
    f_c, w_c = _counter(args.copy_fetch, "FETCH_SIZE"), _counter(args.copy_write, "WRITE_SIZE")
    cf, _ = _match(f_c, args.copy_kernel)
    cw, _ = _match(w_c, args.copy_kernel)
    fscale = args.copy_bytes / (cf * 1024.0)
    wscale = args.copy_bytes / (cw * 1024.0)
    rec_path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(rec_path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    ent = rec.setdefault(args.workload, {})
    lines = [f"# HBM traffic per launch, {args.workload}", "", "Commands (repository root, one MI355X):", "",
             "```", "cd /tmp && export TMPDIR=/tmp && cd -"] + args.cmd + ["```", "",
             f"Copy calibration: `{args.copy_kernel}` moving {args.copy_bytes} bytes reads "
             f"FETCH_SIZE {cf:.0f} KiB and WRITE_SIZE {cw:.0f} KiB per dispatch; scale factors "
             f"{fscale:.4f} (fetch) and {wscale:.4f} (write).", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes per launch |",
             "|---|---:|---:|---:|---:|"]
    for k in args.kernels:
        h = kernel_hash(k)
        fv, nf = _match(f_k, k)
        wv, _ = _match(w_k, k)
        b = fv * 1024.0 * fscale + wv * 1024.0 * wscale
        ent[k] = {"bytes_per_launch": b, "fetch_kib": fv, "write_kib": wv, "fetch_scale": fscale,
                  "write_scale": wscale, "kernel_hash": h}
        lines.append(f"| `{k}` | {nf} | {fv:.0f} | {wv:.0f} | {b:.4g} |")
    with open(rec_path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out} and {rec_path}")


def counters(args):
    path = _one(args.dir, "*counter_collection.csv")
    vals, dur = {}, {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = _fname(r["Kernel_Name"])
            if k in args.kernels:
                vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                dur.setdefault(k, {})[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    for k, d in dur.items():
        vals[k]["duration_s"] = list(d.values())
    names = sorted({c for d in vals.values() for c in d})
    lines = [f"# {args.title}", "", "Command (repository root, one MI355X):", "", "```",
             "cd /tmp && export TMPDIR=/tmp && cd -", args.cmd, "```", ""]
    if args.note:
        lines += [args.note, ""]
    lines += [f"Source: `{os.path.basename(path)}`; median over the dispatches of each kernel.", "",
              "| counter | " + " | ".join(f"`{k}`" for k in args.kernels) + " |",
              "|---|" + "---:|" * len(args.kernels)]
    med = {k: {c: statistics.median(v) for c, v in vals.get(k, {}).items()} for k in args.kernels}
    lines.append("| dispatches | " + " | ".join(str(len(next(iter(vals[k].values())))) if k in vals else "0"
                                              for k in args.kernels) + " |")
    for c in names:
        lines.append(f"| {c} | " + " | ".join(f"{med[k][c]:.4g}" if c in med[k] else "" for k in args.kernels) + " |")

    def ratio(k, a, b, scale=1.0):
        m = med[k]
        return f"{scale * m[a] / m[b]:.3f}" if a in m and b in m and m[b] else ""
    derived = [
        ("engine clock, GHz: GRBM_GUI_ACTIVE / 8 XCDs / dispatch duration",
         lambda k: ratio(k, "GRBM_GUI_ACTIVE", "duration_s", 1.0 / 8 / 1e9)),
        ("MFMA busy per SIMD cycle: SQ_VALU_MFMA_BUSY_CYCLES x 8 / (GRBM_GUI_ACTIVE x 1024)",
         lambda k: ratio(k, "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", 8.0 / 1024.0)),
        ("co-executing share of MFMA busy: SQ_VALU_MFMA_COEXEC_CYCLES / SQ_VALU_MFMA_BUSY_CYCLES",
         lambda k: ratio(k, "SQ_VALU_MFMA_COEXEC_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES")),
        ("vector instructions per matrix instruction, the matrix one included: SQ_INSTS_VALU / SQ_INSTS_MFMA",
         lambda k: ratio(k, "SQ_INSTS_VALU", "SQ_INSTS_MFMA")),
        ("other vector instructions per matrix instruction: (SQ_INSTS_VALU - SQ_INSTS_MFMA) / SQ_INSTS_MFMA",
         lambda k: (f"{med[k]['SQ_INSTS_VALU'] / med[k]['SQ_INSTS_MFMA'] - 1.0:.3f}"
                    if med[k].get("SQ_INSTS_MFMA") else "")),
        ("LDS instructions per matrix instruction: SQ_INSTS_LDS / SQ_INSTS_MFMA",
         lambda k: ratio(k, "SQ_INSTS_LDS", "SQ_INSTS_MFMA")),
    ]
    lines += ["", "| derived | " + " | ".join(f"`{k}`" for k in args.kernels) + " |",
              "|---|" + "---:|" * len(args.kernels)]
    for label, fn in derived:
        lines.append(f"| {label} | " + " | ".join(fn(k) for k in args.kernels) + " |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="Kernel statistics")
    s.add_argument("--note", default="")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("out")
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="Counters")
    c.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--workload", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer")
    t.add_argument("--kernels", nargs="+", required=True)
    t.add_argument("--cmd", nargs="+", required=True)
    t.add_argument("--out", required=True)
    args = ap.parse_args()
    {"stats": stats, "counters": counters, "traffic": traffic}[args.what](args)


if __name__ == "__main__":
    main()
