"""HBM traffic per kernel launch from rocprofv3 counter summaries committed under profiles/.

A summary file profiles/hbm_counters_<workload>.json holds, per kernel, FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) from two `rocprofv3 --pmc` runs, the same counters for a
plain device-to-device copy of known size (the calibration factor), and a hash of the
kernel sources the counters were taken on.  traffic_for() returns the calibrated bytes
per launch only while the sources are unchanged.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
KERNEL_SOURCES = ("csrc/kernels.hip", "csrc/kernels.hpp", "csrc/fft_core.hpp")


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str = "N4095"):
    path = os.path.join(_ROOT, "profiles", f"hbm_counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def parse_counter_csv(path: str, counter: str) -> dict:
    """{kernel_name: mean counter value per dispatch} from a rocprofv3 counter_collection.csv."""
    import csv
    acc: dict = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            acc.setdefault(name, []).append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def find_csv(directory: str, suffix: str = "counter_collection.csv") -> str:
    hits = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return sorted(hits)[-1]
