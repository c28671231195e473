"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2607_26901_amd.profiling --stats STATS.csv \\
        --fetch FETCH.csv --write WRITE.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --copy-mib 512 --occupancy OCC.csv --source paper_2607_26901_amd/csrc/k_broadphase.hip ... \\
        --bench BENCH.json --command "..." --out profiles/c1_kernels.md

* STATS.csv: `rocprofv3 --kernel-trace --stats --output-format csv` kernel
  statistics (per-kernel calls and durations);
* FETCH.csv / WRITE.csv: `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
  counter collections (KiB per dispatch) of the same workload;
* CF.csv / CW.csv: the same counters for a plain device copy of --copy-mib MiB
  (`bench.py --copy-calibration MIB`), which gives the scale from counter
  KiB to bytes actually moved;
* OCC.csv: `rocprofv3 --pmc OccupancyPercent` (waves resident as a share of
  the maximum, per dispatch).

The summary records every kernel's calls, durations, copy-scaled HBM bytes per
dispatch and occupancy, the SHA-256 of the kernel sources and the speed knobs;
`bench.py` uses the traffic figures only while those are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    m = re.search(r"\b(k_\w+)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:40]


def kernel_stats(path: str) -> list[dict]:
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append({"name": short_name(r["Name"]), "calls": int(r["Calls"]),
                         "avg_us": float(r["AverageNs"]) / 1e3, "total_ms": float(r["TotalDurationNs"]) / 1e6,
                         "pct": float(r["Percentage"])})
    rows.sort(key=lambda r: -r["total_ms"])
    return rows


def counter_per_dispatch(path: str) -> dict:
    """kernel -> (dispatches, mean counter value) from a counter-collection CSV."""
    acc = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def copy_scale(path: str, mib: int) -> float:
    """Bytes moved per counter KiB, from the largest dispatch of a copy run."""
    best = 0.0
    with open(path) as f:
        for r in csv.DictReader(f):
            best = max(best, float(r["Counter_Value"]))
    return (mib * (1 << 20)) / best if best > 0 else float("nan")


def sha256(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def knobs_key(t: dict) -> str:
    """The speed knobs a profile was taken with, as one comparable string."""
    key = f"cell_scale={float(t['cell_scale']):.3f} pair_split={int(t['pair_split'])} " \
          f"pair_reuse={int(t.get('pair_reuse', 1))} pair_skin={int(t.get('pair_skin', 0))}"
    if int(t.get("broad_phase", 0)):
        key += f" broad_phase={int(t['broad_phase'])}"
    if int(t.get("direct_regions", 0)):
        key += f" direct_regions={int(t['direct_regions'])}"
    return key


def read_summary(path: str) -> dict:
    """Machine-readable `key: value` lines of a summary written by main()."""
    out = {}
    try:
        with open(path) as f:
            for line in f:
                m = re.match(r"^- `(\w+)`: `([^`]*)`", line.strip())
                if m:
                    out[m.group(1)] = m.group(2)
    except OSError:
        pass
    return out


def occupancy_per_dispatch(path: str) -> dict:
    """kernel -> mean of a per-dispatch occupancy counter (e.g. OccupancyPercent)."""
    return {k: v for k, (n, v) in counter_per_dispatch(path).items()}


def read_kernel_summary(path: str) -> dict:
    """The JSON block of a kernel summary written by main()."""
    try:
        text = open(path).read()
    except OSError:
        return {}
    m = re.search(r"```json\n(.*?)\n```", text, flags=re.S)
    return json.loads(m.group(1)) if m else {}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--occupancy", help="rocprofv3 --pmc OccupancyPercent collection of the same workload")
    ap.add_argument("--source", action="append", default=[], help="a kernel source file the figures depend on")
    ap.add_argument("--bench", required=True, help="bench.py JSON line of the profiled command")
    ap.add_argument("--command", action="append", default=[], help="a command that produced the inputs")
    ap.add_argument("--title", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    stats = kernel_stats(a.stats)
    with open(a.bench) as f:
        b = json.loads(f.readline())
    iters_per_step = int(b.get("config", {}).get("iters_per_step", 1))
    calls = {r["name"]: r for r in stats}
    # k_predict runs once per substep: substeps x iterations = iterations profiled
    iterations = calls["k_predict"]["calls"] * iters_per_step if "k_predict" in calls else 0
    fd = counter_per_dispatch(a.fetch) if a.fetch else {}
    wd = counter_per_dispatch(a.write) if a.write else {}
    fs = copy_scale(a.copy_fetch, a.copy_mib) if a.copy_fetch else float("nan")
    ws = copy_scale(a.copy_write, a.copy_mib) if a.copy_write else float("nan")
    occ = occupancy_per_dispatch(a.occupancy) if a.occupancy else {}
    kernels = {}
    for r in stats:
        k = r["name"]
        rec = {"calls": r["calls"], "avg_us": r["avg_us"], "total_ms": r["total_ms"], "pct": r["pct"]}
        if k in fd and k in wd and fs == fs and ws == ws:
            rec["fetch_kib"] = fd[k][1]
            rec["write_kib"] = wd[k][1]
            rec["traffic_bytes"] = fd[k][1] * fs + wd[k][1] * ws
        if k in occ:
            rec["occupancy_pct"] = occ[k]
        kernels[k] = rec
    facts = {"workload": b.get("config", {}).get("workload", ""), "knobs": knobs_key(b.get("tuning", {})),
             "iterations": iterations, "sources": {src: sha256(src) for src in a.source},
             "fetch_scale": fs / 1024 if fs == fs else None, "write_scale": ws / 1024 if ws == ws else None,
             "kernels": kernels}
    lines = [f"# {a.title or 'Kernels of one workload'}", "",
             "Commands (run from the repository root on the GPU host, each under `cd /tmp && export "
             "TMPDIR=/tmp` for rocprofv3; `<out>` is a folder of the caller's choice):", ""]
    lines += [f"    {c}" for c in a.command]
    lines += ["", f"Profiled: {iterations} solver iterations ({iters_per_step} per substep); knobs "
              f"`{facts['knobs']}`.", "",
              "## Kernel statistics and counters (rocprofv3)", "",
              "| kernel | calls | per iteration | avg us | total ms | % | FETCH KiB | WRITE KiB | HBM MB / dispatch "
              "| occupancy % |", "|---|---|---|---|---|---|---|---|---|---|"]
    for r in stats[:20]:
        k = r["name"]
        rec = kernels[k]
        per_it = r["calls"] / iterations if iterations else float("nan")
        tb = rec.get("traffic_bytes")
        lines.append(f"| {k} | {r['calls']} | {per_it:.3f} | {r['avg_us']:.1f} | {r['total_ms']:.2f} | "
                     f"{r['pct']:.1f} | {rec.get('fetch_kib', float('nan')):.1f} | "
                     f"{rec.get('write_kib', float('nan')):.1f} | "
                     f"{(tb / 1e6) if tb is not None else float('nan'):.2f} | "
                     f"{rec.get('occupancy_pct', float('nan')):.1f} |")
    if fs == fs:
        lines += ["", f"HBM bytes per dispatch = FETCH_SIZE KiB x {fs / 1024:.4f} KiB + WRITE_SIZE KiB x "
                  f"{ws / 1024:.4f} KiB: the factors a plain {a.copy_mib} MiB device copy gives on the same "
                  "counters (bytes moved per counted byte)."]
    rl = b.get("stage_rooflines", {})
    if rl:
        lines += ["", "## The bench line's stage rooflines of the same configuration", "",
                  "| stage | us per iteration (HIP events) | algorithmic bytes | achieved GB/s | fraction of 8 TB/s |",
                  "|---|---|---|---|---|"]
        for st, r in rl.items():
            lines.append(f"| {st} | {r['us_per_iteration']:.1f} | {r['algorithmic_bytes']:.0f} | "
                         f"{r['achieved']:.1f} | {r['frac']:.4f} |")
    lines += ["", "## Figures read by bench.py", "", "```json", json.dumps(facts, indent=1, sort_keys=True), "```"]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
