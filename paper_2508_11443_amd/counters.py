"""Per-kernel HBM traffic from rocprofv3 counter runs.

Two runs of the benchmark under ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``
(``--output-format csv``, bench option ``--copy-calibration`` so that each run starts with
one device copy of exactly 1 GiB) give KiB per dispatch.  Each counter is scaled by what it
reads for that copy (1 GiB read, 1 GiB written), and the per-launch medians of the library's
kernels at the benchmark's grid size are written to ``profiles/traffic.json`` together with
a hash of the kernel's source file, so that ``bench.py`` reports the traffic only while the
kernel is unchanged.

    python -m paper_2508_11443_amd.counters FETCH.csv WRITE.csv profiles/traffic.json

A kernel-trace run (``rocprofv3 --kernel-trace --stats --output-format csv``) is turned
into a markdown table of per-kernel dispatch durations and resources with

    python -m paper_2508_11443_amd.counters trace KERNEL_TRACE.csv

and any counter run (for instance the SQ instruction counters) into a table with

    python -m paper_2508_11443_amd.counters table COUNTER_COLLECTION.csv

What one counted read request of the L2 moves is measured on the random-read probe: the
GPU program ``python -m paper_2508_11443_amd.counters run-probe`` (run under rocprofv3
--pmc) reads 16, 32, 64 and 128 contiguous bytes at uniform random places, and

    python -m paper_2508_11443_amd.counters probe-table RUN1.csv [RUN2.csv ...]

tabulates the counters per dispatch and per read.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GIB = 1 << 30

# timing name used by the library's event timer -> (kernel, as its demangled name reads
# without "void ", "fks::", argument list and spaces; source file)
KERNELS = {
    "fks_lookup_u64": ("k_lookup_u64<true,true,false>", "paper_2508_11443_amd/csrc/lookup.hip"),
    "fks_part_scatter": ("k_dscatter<false,12u,1024u,true>", "paper_2508_11443_amd/csrc/partition.hip"),
    "fks_part_final": ("k_pfinal<false,false,false,true>", "paper_2508_11443_amd/csrc/partition.hip"),
}


def src_sha(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "").replace("fks::", "").replace(" ", "")


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _calibration(rows, name):
    # the 1 GiB copy: the largest copy dispatch of the run
    vals = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"] or
            "copy" in r["Kernel_Name"].lower()]
    big = max(vals)
    return GIB / (big * 1024.0)


def summarize(fetch_csv: str, write_csv: str):
    fr, wr = _rows(fetch_csv), _rows(write_csv)
    sf, sw = _calibration(fr, "FETCH_SIZE"), _calibration(wr, "WRITE_SIZE")
    out = {}
    for timing_name, (sym, src) in KERNELS.items():
        def per_launch(rows):
            mine = [r for r in rows if _short(r["Kernel_Name"]) == sym]
            if not mine:
                return None
            # the benchmark's own launches are the largest grids of this kernel
            gmax = max(int(r["Grid_Size"]) for r in mine)
            return statistics.median(float(r["Counter_Value"]) * 1024.0 for r in mine
                                     if int(r["Grid_Size"]) == gmax)
        f, w = per_launch(fr), per_launch(wr)
        if f is None or w is None:
            continue
        out[timing_name] = {"source_sha": src_sha(src), "source": src,
                            "fetch_bytes_per_launch": round(f * sf), "write_bytes_per_launch": round(w * sw),
                            "hbm_bytes_per_launch": round(f * sf + w * sw),
                            "fetch_scale": round(sf, 4), "write_scale": round(sw, 4)}
    return out


def trace_table(trace_csv: str) -> str:
    """Per library kernel: dispatches, average / min / max duration (us), registers, LDS,
    scratch."""
    rows = _rows(trace_csv)
    by = {}
    for r in rows:
        if "fks::" not in r["Kernel_Name"]:
            continue   # the harness's own torch kernels
        name = _short(r["Kernel_Name"])
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        ent = by.setdefault(name, {"d": [], "vgpr": r.get("Arch_VGPR_Count", r.get("VGPR_Count", "")),
                                   "sgpr": r.get("SGPR_Count", ""), "lds": r.get("LDS_Block_Size", ""),
                                   "scratch": r.get("Scratch_Size", ""),
                                   "grid": r.get("Grid_Size", r.get("Grid_Size_X", ""))})
        ent["d"].append(us)
    lines = ["| kernel | calls | avg us | min us | max us | grid | VGPR | SGPR | LDS B | scratch B |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for name, e in sorted(by.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = e["d"]
        lines.append(f"| {name} | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} | {e['grid']} | "
                     f"{e['vgpr']} | {e['sgpr']} | {e['lds']} | {e['scratch']} |")
    return "\n".join(lines)


def counter_table(csv_path: str) -> str:
    """Per library kernel and launch size: every counter of a --pmc run, averaged over the
    launches, with per-wave figures for the SQ instruction and cycle counters."""
    rows = [r for r in _rows(csv_path) if "fks::" in r["Kernel_Name"]]
    by = {}
    for r in rows:
        key = (_short(r["Kernel_Name"]), int(r["Grid_Size"]))
        ent = by.setdefault(key, {})
        ent.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for e in by.values() for c in e})
    lines = ["| kernel | grid | " + " | ".join(names) + " | per wave: " +
             ", ".join(n for n in names if n != "SQ_WAVES") + " |",
             "|---|---|" + "---|" * (len(names) + 1)]
    for (name, grid), e in sorted(by.items(), key=lambda kv: -kv[0][1]):
        avg = {c: sum(v) / len(v) for c, v in e.items()}
        waves = avg.get("SQ_WAVES", 0.0)
        per = ", ".join(f"{avg[c] / waves:.0f}" for c in names if c != "SQ_WAVES" and c in avg) if waves else ""
        lines.append(f"| {name} | {grid} | " + " | ".join(f"{avg.get(c, float('nan')):.4g}" for c in names) +
                     f" | {per} |")
    return "\n".join(lines)


PROBE_READS = 1 << 27
PROBE_WIDTHS = (16, 32, 64, 128)


def run_probe():
    """GPU program for counter runs over the random-read probe: one 1 GiB device copy (known
    bytes, for scaling), then fks_probe_random_reads at every width: 2^27 reads from a 2 GiB
    buffer, each width launched twice (warm-up and timed) with its own kernel instance."""
    import torch
    from . import fks
    dev = torch.device("cuda:0")
    src = torch.ones(1 << 27, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    for w in PROBE_WIDTHS:
        ms = fks.fks_probe_random_reads(2 << 30, PROBE_READS, w)
        print(f"probe width {w} B: {PROBE_READS / (ms * 1e-3) / 1e9:.2f} G reads/s", flush=True)


def probe_table(*csv_paths) -> str:
    """Per probe width: every counter of the given --pmc runs per dispatch and per read, and
    the same counters for the 1 GiB copy per 128-byte line it streams."""
    per = {}
    copy = {}
    for path in csv_paths:
        for r in _rows(path):
            name, v = r["Kernel_Name"], float(r["Counter_Value"])
            if "k_probe_random" in name:
                vec = int(_short(name).split("<")[1].rstrip(">"))
                per.setdefault(16 * vec, {}).setdefault(r["Counter_Name"], []).append(v)
            elif "copy" in name.lower():
                copy.setdefault(r["Counter_Name"], []).append(v)
    names = sorted({c for e in per.values() for c in e})
    lines = ["| reads of | " + " | ".join(f"{c} / dispatch" for c in names) + " | " +
             " | ".join(f"{c} / read" for c in names) + " |", "|---|" + "---|" * (2 * len(names))]
    for w in sorted(per):
        avg = {c: statistics.median(v) for c, v in per[w].items()}
        lines.append(f"| {w} B | " + " | ".join(f"{avg.get(c, float('nan')):.4g}" for c in names) + " | " +
                     " | ".join(f"{avg.get(c, float('nan')) / PROBE_READS:.3f}" for c in names) + " |")
    if copy:
        lines_gib = GIB // 128
        big = {c: max(v) for c, v in copy.items()}
        lines.append(f"| 1 GiB copy (per 128-B line read) | " + " | ".join(f"{big.get(c, float('nan')):.4g}"
                                                                           for c in names) + " | " +
                     " | ".join(f"{big.get(c, float('nan')) / lines_gib:.3f}" for c in names) + " |")
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[1] == "run-probe":
        run_probe()
        return
    if len(argv) >= 3 and argv[1] == "probe-table":
        print(probe_table(*argv[2:]))
        return
    if len(argv) >= 3 and argv[1] == "trace":
        print(trace_table(argv[2]))
        return
    if len(argv) >= 3 and argv[1] == "table":
        print(counter_table(argv[2]))
        return
    fetch_csv, write_csv, dest = argv[1:4]
    data = summarize(fetch_csv, write_csv)
    with open(dest, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(data, indent=1))


if __name__ == "__main__":
    main(sys.argv)
