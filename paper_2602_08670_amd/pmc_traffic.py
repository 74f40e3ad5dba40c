"""Per-launch HBM traffic of the stage kernels from two rocprofv3 counter runs.

rocprofv3 reports FETCH_SIZE and WRITE_SIZE in KiB per dispatch.  Their
units are not taken on trust: each counter is scaled by what it reads for a
kernel of known traffic in the same process.  The bench run started with
--calib-copy-mb M first fills an M-MiB buffer (torch's fill kernel: writes M
MiB) and copies it (the runtime's copy kernel: reads and writes M MiB).  On
MI355X the fetch counter reads half the copy's bytes and the write counter
reads them exactly, so the factors come out near 2 and 1.

    python -m paper_2602_08670_amd.pmc_traffic FETCH_DIR WRITE_DIR --calib-mb 256 --out FILE

FETCH_DIR / WRITE_DIR hold the *_counter_collection.csv of a
`rocprofv3 --pmc FETCH_SIZE` and a `rocprofv3 --pmc WRITE_SIZE` run of the
same command.  The output records the scale factors, the mean scaled bytes
per dispatch of each stage kernel, and the SHA-256 of the kernel sources the
counters were taken on (bench.py reports the traffic only while it matches).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/fv_kernels.hip", "csrc/fv_device.hpp", "csrc/fv_internal.hpp")


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_kernel(rows, counter):
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def summarize(fetch_dir: str, write_dir: str, calib_mb: int, match: str = "batch_stage_one_kernel<float, 0, true"):
    calib_kib = calib_mb * 1024.0
    fetch = _per_kernel(_rows(fetch_dir), "FETCH_SIZE")
    write = _per_kernel(_rows(write_dir), "WRITE_SIZE")
    # calibration: the largest copy kernel reads calib_kib; the largest fill writes calib_kib
    copy_fetch = max(v for k, vals in fetch.items() if "copyBuffer" in k for _, v in vals)
    fill_write = max(v for k, vals in write.items() if "FillFunctor" in k for _, v in vals)
    fs, ws = calib_kib / copy_fetch, calib_kib / fill_write
    res = {"kernel_sources_sha256": kernel_sources_sha256(), "calib_mib": calib_mb,
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4), "kernels": {}}
    for name in sorted(set(fetch) | set(write)):
        if match not in name:
            continue
        f = statistics.mean(v for _, v in fetch.get(name, [(0, 0.0)]))
        w = statistics.mean(v for _, v in write.get(name, [(0, 0.0)]))
        res["kernels"][name] = {"dispatches": len(fetch.get(name, [])), "fetch_kib_raw": round(f, 1),
                                "write_kib_raw": round(w, 1), "bytes": round((f * fs + w * ws) * 1024)}
    if res["kernels"]:
        res["bytes_per_launch"] = round(statistics.mean(k["bytes"] for k in res["kernels"].values()))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--calib-mb", type=int, required=True)
    ap.add_argument("--match", default="batch_stage_one_kernel<float, 0, true")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = summarize(a.fetch_dir, a.write_dir, a.calib_mb, a.match)
    txt = json.dumps(res, indent=1)
    print(txt)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
