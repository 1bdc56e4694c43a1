"""HBM traffic per launch from rocprofv3 counter runs.

Reads the counter-collection CSVs of two `rocprofv3 --pmc` runs of the same command (one
with FETCH_SIZE, one with WRITE_SIZE; both in KiB per dispatch) and the same two runs of a
plain copy kernel of known size (`qimax_copy_probe`), and writes, per kernel, the average
HBM bytes per launch: (FETCH_SIZE x f_fetch + WRITE_SIZE x f_write) x 1024, where the
factors f scale each counter so that the copy kernel reads and writes exactly its bytes.

    python -m paper_2505_03307_amd.hbm_traffic --workload c2 --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --copy-bytes B -o profiles/traffic.json

The output holds one object per workload (merged into an existing file), keyed by the kernel
names the library's profiler uses; every entry carries a hash of the kernel sources: a
reader ignores an entry whose kernels have changed since.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))

# library profiler name -> pattern of the kernel symbol(s) it covers
KERNELS = {
    "count": r"\bk_count_scan",
    "count_expand": r"\bk_count_expand",
    "expand": r"\bk_expand",
    "sort_hist": r"\bk_sort_(upsweep|hist)",
    "sort_scatter": r"\bk_sort_scatter",
    "chunk_sort": r"\bk_chunk_sort",
    "dense_merge": r"\bk_dense_(scatter|compact)",
    "chunk_finish": r"\bk_chunk_(publish|compact)\b",
    # with truncated kernel names (rocprofv3 -T) k_merge counts as the writing merge, the one
    # the benchmark runs
    "merge_count": r"\bk_merge<[^,]+, [^,]+, 0>",
    "merge_write": r"\bk_merge<[^,]+, [^,]+, [12]>|\bk_merge$",
    "copy": r"\bk_copy_u64",
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "qimax_internal.h"):
        with open(os.path.join(_HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counter(d: str, counter: str):
    """{kernel symbol: [value per dispatch]} from the counter CSVs under d."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def per_kernel(values, pattern: str):
    rx = re.compile(pattern)
    vals = [v for k, vs in values.items() if rx.search(k) for v in vs]
    return vals


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True, help="bytes one copy launch reads (and writes)")
    ap.add_argument("-o", "--out", required=True)
    ap.add_argument("--workload", required=True, help="name of the profiled workload (e.g. c2, hea-fp64)")
    a = ap.parse_args(argv)
    fetch, write = read_counter(a.fetch, "FETCH_SIZE"), read_counter(a.write, "WRITE_SIZE")
    cf = per_kernel(read_counter(a.copy_fetch, "FETCH_SIZE"), KERNELS["copy"])
    cw = per_kernel(read_counter(a.copy_write, "WRITE_SIZE"), KERNELS["copy"])
    if not cf or not cw:
        raise SystemExit("copy kernel not found in the calibration runs")
    # median over the copy launches; KiB -> bytes
    f_fetch = a.copy_bytes / (sorted(cf)[len(cf) // 2] * 1024.0)
    f_write = a.copy_bytes / (sorted(cw)[len(cw) // 2] * 1024.0)
    out = {"_calibration": {"copy_bytes": a.copy_bytes, "fetch_factor": round(f_fetch, 4),
                            "write_factor": round(f_write, 4)}}
    src = kernel_source_hash()
    for name, pat in KERNELS.items():
        if name == "copy":
            continue
        fv, wv = per_kernel(fetch, pat), per_kernel(write, pat)
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024.0 * f_fetch
        wb = sum(wv) / len(wv) * 1024.0 * f_write
        out[name] = {"launches": len(fv), "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                     "bytes_per_launch": round(fb + wb), "source_hash": src}
    allw = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            allw = json.load(fh)
        if "_calibration" in allw:  # an older single-workload file
            allw = {}
    allw[a.workload] = out
    with open(a.out, "w") as fh:
        json.dump(allw, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(out, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()
