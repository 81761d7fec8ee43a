"""HBM traffic per kernel launch from rocprofv3 counter runs.

Two runs of the same program, one with ``--pmc FETCH_SIZE`` and one with
``--pmc WRITE_SIZE`` (a run collects one of them; together they exceed the L2
counter block), each write a ``*_counter_collection.csv`` with one row per
dispatch.  Both counters are derived values in KiB; each is scaled by the
factor that maps its reading on a plain 1 GiB device-to-device copy (the
runtime's ``__amd_rocclr_copyBuffer``, which reads and writes exactly 1 GiB)
onto 1 GiB.  The result, per kernel, is the HBM bytes one launch moves,
recorded with a hash of the HIP sources it was taken on: a record whose hash
no longer matches the sources describes other kernels and is not reported.

    python -m paper_1810_11765_amd.counters FETCH.csv WRITE.csv OUT.json
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 1 << 30
CALIB_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_GRID = 131072              # the 1 GiB copy's dispatch (other copies are smaller)
SWEEP_GRID = 2097152             # the 2^21-block sweep's dispatch in the bench


def kernel_source_hash() -> str:
    """Hash of the HIP sources; counter figures taken on other sources are stale."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def short_name(kernel: str, grid: int) -> str:
    """``smmo::k_doall<smmo::MLifeCommit, false, false>`` or ``void
    k_doall<MLifeCommit>(DevHeap, ...)`` -> ``k_doall<MLifeCommit>`` (the
    profiler prints either form); the streaming sweep at the bench's
    2^21-block shape gets ``@2^21``."""
    k = kernel.replace("smmo::", "")
    if k.startswith("void "):
        k = k[5:]
    depth = 0
    for i, c in enumerate(k):               # cut the parameter list at template depth 0
        depth += (c == "<") - (c == ">")
        if c == "(" and depth == 0 and i > 0:
            k = k[:i]
            break
    k = re.sub(r"(, (true|false))+>", ">", k)
    if k.startswith("k_doall_axpy<") and grid == SWEEP_GRID:
        k += "@2^21"
    return k


def read(path: str, counter: str):
    """{kernel short name: [value per dispatch]} and the calibration copy's values."""
    per, calib = {}, []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            grid, v = int(row["Grid_Size"]), float(row["Counter_Value"])
            if row["Kernel_Name"] == CALIB_KERNEL and grid == CALIB_GRID:
                calib.append(v)
            per.setdefault(short_name(row["Kernel_Name"], grid), []).append(v)
    return per, calib


def traffic(fetch_csv: str, write_csv: str) -> dict:
    fetch, fcal = read(fetch_csv, "FETCH_SIZE")
    write, wcal = read(write_csv, "WRITE_SIZE")
    if not fcal or not wcal:
        raise SystemExit("no 1 GiB calibration copy in the counter runs (run the program with --calib-copy)")
    ff = CALIB_BYTES / 1024 / statistics.median(fcal)
    wf = CALIB_BYTES / 1024 / statistics.median(wcal)
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if k.startswith("__amd") or k.startswith("at::"):
            continue
        fk, wk = statistics.fmean(fetch[k]), statistics.fmean(write[k])
        kernels[k] = {"fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1), "dispatches": len(fetch[k]),
                      "bytes_per_launch": int(round((fk * ff + wk * wf) * 1024))}
    return {"source_sha256": kernel_source_hash(),
            "how": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE (separate runs) of python3 bench.py "
                   "--no-cpu-baseline --no-batch --calib-copy; per-dispatch KiB averaged per kernel, times the "
                   "factor that maps the 1 GiB runtime copy (copyBuffer, grid 131072) onto 1 GiB read + 1 GiB written",
            "fetch_factor": round(ff, 5), "write_factor": round(wf, 5),
            "calib_fetch_kib": statistics.median(fcal), "calib_write_kib": statistics.median(wcal),
            "kernels": kernels}


def main(argv):
    if len(argv) != 4:
        raise SystemExit(__doc__)
    rec = traffic(argv[1], argv[2])
    with open(argv[3], "w") as f:
        json.dump(rec, f, indent=1)
    for k, v in rec["kernels"].items():
        print(f"{k:48s} {v['dispatches']:7d} {v['fetch_kib_raw']:12.1f} {v['write_kib_raw']:12.1f} "
              f"{v['bytes_per_launch']:15d}")


if __name__ == "__main__":
    main(sys.argv)
