"""Summaries of rocprofv3 output for the committed profile notes.

    python -m paper_2606_20426_amd.profiling stats  STATS_CSV  OUT.md --command "..."
    python -m paper_2606_20426_amd.profiling traffic FETCH_CSV WRITE_CSV OUT.md \
        --probe-mib 512 --kernel cg_spmv --workload batch60 --command-fetch "..." --command-write "..."

`stats` turns a `--kernel-trace --stats` kernel_stats CSV into a table of
calls, average and total duration per kernel.

`counters` turns one `--pmc` counter CSV (any counters) into a table of
per-dispatch averages per kernel.

`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` counter CSVs
(KiB per dispatch) into HBM bytes per launch.  The counters are scaled by
what they read for a device copy of known size run in the same process
(`bench.py --copy-probe MiB`: the largest copy dispatches read and write
exactly that many bytes).  The note records a hash of the kernel sources so
that a reader can tell whether the figures still describe the kernels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_2606_20426_amd/csrc/kernels.hip", "paper_2606_20426_amd/csrc/tc_device.h")
# library kernel id -> substring of the compiled kernel's name
KERNEL_SYMBOL = {
    "cg_spmv": "k_cg_spmv",
    "cg_update": "k_cg_update",
    "element": "k_element",
    "asm_diag": "k_asm_diag",
    "asm_off": "k_asm_off",
    "energy": "k_energy",
    "sigma": "k_sigma",
    "traction": "k_traction",
}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_sources_hash(root=ROOT):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name):
    base = name.split("(")[0]
    return base.replace("void ", "").replace("tc::", "")


def stats_table(path, top=30):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | avg µs | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append("| `%s` | %d | %.2f | %.1f | %.1f |" % (
            short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, 100.0 * float(r["TotalDurationNs"]) / total))
    return out, total


def per_kernel_kib(path):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return acc


def copy_factor(acc, probe_mib):
    """bytes actually moved by the probe copy / bytes the counter reports."""
    vals = acc.get(COPY_KERNEL, [])
    if not vals:
        raise SystemExit("no copy dispatches in the counter file")
    top = max(vals)
    probe = [v for v in vals if v > 0.5 * top]
    kib = sum(probe) / len(probe)
    return probe_mib * 1024.0 / kib, kib, len(probe)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("stats_csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="Kernel trace statistics")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="Counters per dispatch")
    c.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--probe-mib", type=int, required=True)
    t.add_argument("--kernel", default="cg_spmv")
    t.add_argument("--workload", default="batch60")
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    a = ap.parse_args(argv)

    if a.cmd == "stats":
        table, total = stats_table(a.stats_csv)
        lines = [f"# {a.title}", "", "Command (from the repository root, after `cd /tmp && export TMPDIR=/tmp`):", "",
                 "```", a.command, "```", "",
                 f"- kernel_sources_sha256: `{kernel_sources_hash()}`",
                 f"- total kernel time: {total / 1e6:.1f} ms", ""] + table + [""]
        open(a.out, "w").write("\n".join(lines))
        return

    if a.cmd == "counters":
        acc = collections.defaultdict(lambda: collections.defaultdict(list))
        calls = collections.Counter()
        for r in csv.DictReader(open(a.csv)):
            name = short_name(r["Kernel_Name"])
            acc[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
        names = sorted({c for d in acc.values() for c in d})
        for k, d in acc.items():
            calls[k] = max(len(v) for v in d.values())
        lines = [f"# {a.title}", "", "Command (from the repository root, after `cd /tmp && export TMPDIR=/tmp`):", "",
                 "```", a.command, "```", "",
                 f"- kernel_sources_sha256: `{kernel_sources_hash()}`",
                 "- values: averages over the kernel's dispatches of what rocprofv3 reports per dispatch", "",
                 "| kernel | dispatches | " + " | ".join(names) + " |",
                 "|---|---:|" + "---:|" * len(names)]
        for k, _ in calls.most_common(a.top):
            d = acc[k]
            vals = [("%.4g" % (sum(d[n]) / len(d[n]))) if d.get(n) else "" for n in names]
            lines.append(f"| `{k}` | {calls[k]} | " + " | ".join(vals) + " |")
        lines.append("")
        open(a.out, "w").write("\n".join(lines))
        return

    fetch = per_kernel_kib(a.fetch_csv)
    write = per_kernel_kib(a.write_csv)
    ff, fkib, fn = copy_factor(fetch, a.probe_mib)
    wf, wkib, wn = copy_factor(write, a.probe_mib)
    sym = KERNEL_SYMBOL[a.kernel]
    rows = []
    for name in sorted(set(fetch) | set(write)):
        if COPY_KERNEL in name:
            continue
        fv, wv = fetch.get(name, []), write.get(name, [])
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024.0 * ff
        wb = sum(wv) / len(wv) * 1024.0 * wf
        rows.append((short_name(name), len(fv), fb, wb, name))
    rows.sort(key=lambda r: -(r[2] + r[3]) * r[1])
    dom = [r for r in rows if sym in r[4]]
    if not dom:
        raise SystemExit(f"kernel {a.kernel} not found")
    d = dom[0]
    lines = [f"# HBM traffic per launch, {a.workload}", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two counter passes of the same command,",
             f"scaled by what each counter reads for a {a.probe_mib} MiB device copy run first in the same",
             "process (`--copy-probe`): the copy reads and writes exactly that many bytes.", "",
             "Commands (from the repository root, after `cd /tmp && export TMPDIR=/tmp`):", "",
             "```", a.command_fetch, a.command_write, "```", "",
             f"- workload: `{a.workload}`",
             f"- kernel: `{a.kernel}`",
             f"- kernel_sources_sha256: `{kernel_sources_hash()}`",
             f"- copy_fetch_kib: {fkib:.1f} over {fn} dispatches (factor {ff:.4f})",
             f"- copy_write_kib: {wkib:.1f} over {wn} dispatches (factor {wf:.4f})",
             f"- dispatches: {d[1]}",
             f"- fetch_bytes_per_launch: {d[2]:.0f}",
             f"- write_bytes_per_launch: {d[3]:.0f}",
             f"- traffic_bytes_per_launch: {d[2] + d[3]:.0f}", "",
             "| kernel | dispatches | fetch MB/launch | write MB/launch |", "|---|---:|---:|---:|"]
    for r in rows[:16]:
        lines.append("| `%s` | %d | %.2f | %.2f |" % (r[0], r[1], r[2] / 1e6, r[3] / 1e6))
    lines.append("")
    open(a.out, "w").write("\n".join(lines))


if __name__ == "__main__":
    main()
