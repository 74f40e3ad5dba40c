"""Mean per-dispatch hardware counters of the kernels of one rocprofv3 --pmc
run, for dispatches of a given grid size (the timed workload's launches).

    python -m paper_2602_08670_amd.pmc_counters DIR --match batch_stage_kernel --grid 524288

DIR holds the *_counter_collection.csv of the run.  Prints one JSON object:
per kernel name, the dispatch count and the mean of every counter.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics


def collect(d: str, match: str, grid: int):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    acc = {}
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            if match not in r["Kernel_Name"] or (grid and int(r["Grid_Size"]) != grid):
                continue
            k = acc.setdefault(r["Kernel_Name"], {})
            k.setdefault(r["Counter_Name"], {})[r["Dispatch_Id"]] = float(r["Counter_Value"])
    out = {}
    for name, counters in acc.items():
        out[name] = {"dispatches": max(len(v) for v in counters.values())}
        for c, vals in sorted(counters.items()):
            out[name][c] = round(statistics.mean(vals.values()), 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--match", default="batch_stage_kernel")
    ap.add_argument("--grid", type=int, default=0)
    a = ap.parse_args()
    print(json.dumps(collect(a.dir, a.match, a.grid), indent=1))


if __name__ == "__main__":
    main()
