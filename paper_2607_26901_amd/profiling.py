"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2607_26901_amd.profiling --stats STATS.csv \\
        --fetch FETCH.csv --write WRITE.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --copy-mib 512 --kernel k_pairs --source paper_2607_26901_amd/csrc/k_broadphase.hip \\
        --bench BENCH.json --command "..." --out profiles/pair_emission_c1.md

* STATS.csv: `rocprofv3 --kernel-trace --stats --output-format csv` kernel
  statistics (per-kernel calls and durations);
* FETCH.csv / WRITE.csv: `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
  counter collections (KiB per dispatch) of the same workload;
* CF.csv / CW.csv: the same counters for a plain device copy of --copy-mib MiB
  (`bench.py --copy-calibration MIB`), which gives the scale from counter
  KiB to bytes actually moved.

The summary records the SHA-256 of the kernel's source file; `bench.py` uses the
traffic figure only while the source is unchanged.
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
    return f"cell_scale={float(t['cell_scale']):.3f} pair_split={int(t['pair_split'])} " \
           f"pair_reuse={int(t.get('pair_reuse', 1))} pair_skin={int(t.get('pair_skin', 0))}"


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


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--kernel", default="k_pairs")
    ap.add_argument("--stage", default="pair_emission",
                    help="bench.py's name of the kernel's stage; the bench figures are recorded only when the "
                         "bench's roofline is for this stage")
    ap.add_argument("--source", required=True)
    ap.add_argument("--bench", help="bench.py JSON line of the same workload")
    ap.add_argument("--command", action="append", default=[], help="a command that produced the inputs")
    ap.add_argument("--title", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    stats = kernel_stats(a.stats)
    lines = [f"# {a.title or a.kernel}", "", "Commands (run from the repository root on the GPU host):", ""]
    lines += [f"    {c}" for c in a.command]
    lines += ["", "## Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in stats[:14]:
        lines.append(f"| {r['name']} | {r['calls']} | {r['avg_us']:.1f} | {r['total_ms']:.2f} | {r['pct']:.1f} |")
    mine = [r for r in stats if r["name"] == a.kernel]
    facts = {"kernel": a.kernel, "source": a.source, "source_sha256": sha256(a.source)}
    if mine:
        facts["rocprof_avg_us"] = f"{mine[0]['avg_us']:.2f}"
    if a.bench:
        with open(a.bench) as f:
            b = json.loads(f.readline())
        rl = b.get("roofline", {})
        if "tuning" in b:
            facts["knobs"] = knobs_key(b["tuning"])
        if rl.get("kernel") == a.stage:
            facts["bench_avg_launch_us"] = f"{rl.get('avg_launch_us', float('nan')):.2f}"
            facts["algorithmic_bytes_per_launch"] = f"{rl.get('algorithmic_bytes', float('nan')):.0f}"
    if a.fetch and a.write and a.copy_fetch and a.copy_write:
        fs, ws = copy_scale(a.copy_fetch, a.copy_mib), copy_scale(a.copy_write, a.copy_mib)
        fd, wd = counter_per_dispatch(a.fetch), counter_per_dispatch(a.write)
        nf, f_kib = fd.get(a.kernel, (0, float("nan")))
        nw, w_kib = wd.get(a.kernel, (0, float("nan")))
        facts.update({"fetch_kib_per_dispatch": f"{f_kib:.1f}", "write_kib_per_dispatch": f"{w_kib:.1f}",
                      "fetch_scale": f"{fs / 1024:.4f}", "write_scale": f"{ws / 1024:.4f}",
                      "traffic_bytes_per_launch": f"{f_kib * fs + w_kib * ws:.0f}",
                      "dispatches_counted": f"{nf}/{nw}"})
        lines += ["", "## HBM traffic per dispatch (rocprofv3 --pmc, separate runs)", "",
                  "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|"]
        for k in sorted(fd, key=lambda k: -fd[k][1])[:10]:
            lines.append(f"| {k} | {fd[k][1]:.1f} | {wd.get(k, (0, float('nan')))[1]:.1f} |")
        lines += ["", f"Scale from a plain {a.copy_mib} MiB device copy: FETCH_SIZE x{fs / 1024:.4f}, "
                  f"WRITE_SIZE x{ws / 1024:.4f} (bytes per counted byte)."]
    lines += ["", "## Figures used by bench.py", ""]
    lines += [f"- `{k}`: `{v}`" for k, v in facts.items()]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
