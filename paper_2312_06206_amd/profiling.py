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


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed: edits to comments or
    layout do not change the compiled kernels, so they keep committed counters valid."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel)) as f:
            h.update(_code_only(f.read()).encode())
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


# the kernels of a step n >= 1 inside a multi-step run, by name prefix and template tail
# kernels of a run of steps (the row transform runs once per run; the state in paired rows)
KERNEL_KEYS = {"rows_fwd": ("rows_fwd_kernel<", ", 0, 0>"), "cols_conv": ("cols_conv_kernel<", ">"),
               "rows_rhs_gs": ("rows_rhs_gs_kernel<", ", 0, 1, 1>"), "cols_gs_fwd": ("cols_gs_fwd_kernel<", ", 1>")}


def kernel_key(name: str, m: int):
    """Step-kernel key of a demangled kernel name for line length m, or None."""
    for key, (head, tail) in KERNEL_KEYS.items():
        if f"{head}{m}{tail}" in name:
            return key
    return None


def _mean_by_kernel(path: str, counter: str, m: int) -> dict:
    """Mean counter value per dispatch of the n >= 1 step kernels of length m."""
    import csv
    acc: dict = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            key = kernel_key(name, m)
            if key:
                acc.setdefault(key, []).append(float(row["Counter_Value"]))
            if "elementwise" in name and "Mul" in name:
                acc.setdefault("_copy", []).append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def write_kernel_stats_summary(stats_csv: str, n: int, out_md: str, command: str,
                               title: str = "") -> dict:
    """Short markdown table of a `rocprofv3 --kernel-trace --stats` kernel_stats.csv: calls,
    average and total duration of every kernel, FP64 step kernels of length n + 1 labelled."""
    import csv
    m = n + 1
    rows = []
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["TotalDurationNs"]),
                         float(r.get("Percentage", 0.0))))
    rows.sort(key=lambda r: -r[3])
    steps = {}
    lines = [f"# Kernel trace, {title or f'S-ADI FP64, N={n}'}", "", "Command (from the repository root):", "",
             "```", command, "```", "",
             "| kernel | step role | calls | avg us | total ms | % |", "|---|---|---|---|---|---|"]
    for name, calls, avg, tot, pct in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("sadi::", "")
        key = kernel_key(name, m) or ""
        if key:
            steps[key] = {"calls": calls, "avg_us": avg / 1e3}
        lines.append(f"| `{short[:70]}` | {key} | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.3f} | {pct:.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return steps


def write_traffic_summary(fetch_dir: str, write_dir: str, calib_fetch_dir: str, calib_write_dir: str,
                          n: int, out_json: str, command: str) -> dict:
    """Combine FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch) of the benchmark and of the
    copy calibration into bytes per launch for each step kernel."""
    m = n + 1
    fetch = _mean_by_kernel(find_csv(fetch_dir), "FETCH_SIZE", m)
    write = _mean_by_kernel(find_csv(write_dir), "WRITE_SIZE", m)
    cf = _mean_by_kernel(find_csv(calib_fetch_dir), "FETCH_SIZE", m)["_copy"]
    cw = _mean_by_kernel(find_csv(calib_write_dir), "WRITE_SIZE", m)["_copy"]
    copy_bytes = float(1 << 30)
    f_fetch = cf * 1024.0 / copy_bytes        # counter bytes per true byte, reads
    f_write = cw * 1024.0 / copy_bytes
    rec = {"workload": f"N{n}", "command": command, "source_hash": source_hash(),
           "calibration": {"copy_bytes": copy_bytes, "fetch_kib_per_copy": cf, "write_kib_per_copy": cw,
                           "fetch_factor": f_fetch, "write_factor": f_write},
           "kernels": {}}
    for k in KERNEL_KEYS:
        if k in fetch and k in write:
            rb = fetch[k] * 1024.0 / f_fetch
            wb = write[k] * 1024.0 / f_write
            rec["kernels"][k] = {"fetch_kib": fetch[k], "write_kib": write[k], "read_bytes": rb,
                                 "write_bytes": wb, "bytes_per_launch": rb + wb}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


VALU_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                 "SQ_INSTS_VALU_FMA_F64")


def write_valu_summary(pmc_dir: str, n: int, out_json: str, command: str) -> dict:
    """Per-dispatch wave-instruction counts of the step kernels from one rocprofv3 --pmc run
    of SQ_WAVES and the SQ_INSTS_VALU family: all VALU instructions and the FP64 add / mul /
    fma ones (each a wave64 instruction)."""
    m = n + 1
    path = find_csv(pmc_dir)
    per = {c: _mean_by_kernel(path, c, m) for c in VALU_COUNTERS}
    rec = {"workload": f"N{n}", "command": command, "source_hash": source_hash(), "kernels": {}}
    for k in KERNEL_KEYS:
        if all(k in per[c] for c in VALU_COUNTERS):
            v = {c: per[c][k] for c in VALU_COUNTERS}
            # FP64 flops: 64 lanes per wave instruction, an fma counts two
            v["fp64_flops"] = 64.0 * (v["SQ_INSTS_VALU_ADD_F64"] + v["SQ_INSTS_VALU_MUL_F64"]
                                      + 2.0 * v["SQ_INSTS_VALU_FMA_F64"])
            rec["kernels"][k] = v
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def write_pmc_summary(pmc_dirs: list, n: int, out_json: str, commands: list) -> dict:
    """Mean per-dispatch value of every counter in one or more rocprofv3 --pmc runs, for the
    step kernels of length n + 1 (one record per kernel, counters merged over the runs)."""
    import csv
    m = n + 1
    rec = {"workload": f"N{n}", "commands": commands, "source_hash": source_hash(), "kernels": {}}
    for d in pmc_dirs:
        acc: dict = {}
        with open(find_csv(d)) as f:
            for row in csv.DictReader(f):
                key = kernel_key(row.get("Kernel_Name", ""), m)
                if key:
                    acc.setdefault((key, row["Counter_Name"]), []).append(float(row["Counter_Value"]))
        for (key, c), v in acc.items():
            rec["kernels"].setdefault(key, {})[c] = sum(v) / len(v)
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def valu_for(kernel: str, workload: str = "N4095"):
    """The committed VALU counts of a step kernel, if taken on the current kernel sources."""
    path = os.path.join(_ROOT, "profiles", f"valu_counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("kernels", {}).get(kernel)


MFMA_PEAK_TFLOPS = {"double": 78.6, "float": 157.3}   # MI355X dense matrix-core peaks


def write_mfma_summary(pmc_dir: str, out_md: str, command: str) -> list:
    """Matrix-core use of every product kernel dispatch in one rocprofv3 --pmc run of
    SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32 (units of 512 flops): dispatches grouped by kernel,
    work-items and flops, with the achieved rate from each dispatch's own start and end times
    against the dense peak of its operand type."""
    import csv
    per: dict = {}
    with open(find_csv(pmc_dir)) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            if "gemm_mfma_kernel" not in name:
                continue
            d = per.setdefault(row["Dispatch_Id"], {"name": name, "items": int(row["Grid_Size"]),
                                                    "ns": float(row["End_Timestamp"]) - float(row["Start_Timestamp"])})
            d[row["Counter_Name"]] = float(row["Counter_Value"])
    groups: dict = {}
    for d in per.values():
        ti = "float" if "gemm_mfma_kernel<float" in d["name"] else "double"
        mops = d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
        flops = 512.0 * mops
        short = d["name"].replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("sadi::", "")
        key = (short, d["items"], round(flops / 1e6))
        g = groups.setdefault(key, {"kernel": short, "type": ti, "work_items": d["items"], "flops": flops,
                                    "calls": 0, "ns": 0.0, "busy": 0.0, "gui": 0.0})
        g["calls"] += 1
        g["ns"] += d["ns"]
        g["busy"] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        g["gui"] += d.get("GRBM_GUI_ACTIVE", 0.0)
    out = []
    for g in groups.values():
        avg_us = g["ns"] / g["calls"] / 1e3
        tf = g["flops"] / (avg_us * 1e-6) / 1e12 if avg_us > 0 else 0.0
        out.append(dict(g, avg_us=avg_us, tflops=tf, frac=tf / MFMA_PEAK_TFLOPS[g["type"]]))
    out.sort(key=lambda g: -g["flops"] * g["calls"])
    lines = ["# Matrix-core use of the product kernels", "", "Command (from the repository root):", "",
             "```", command, "```", "",
             "Rate = flops from SQ_INSTS_VALU_MFMA_MOPS_* (x 512) over each dispatch's own duration in the "
             "counter run; peak = MI355X dense matrix-core rate of the operand type (FP64 78.6, FP32 157.3 "
             "TFLOP/s).", "",
             "| kernel | calls | work-items | GFLOP per call | avg us | TFLOP/s | % of peak |",
             "|---|---|---|---|---|---|---|"]
    for g in out:
        lines.append(f"| `{g['kernel'][:60]}` | {g['calls']} | {g['work_items']} | {g['flops'] / 1e9:.3f} | "
                     f"{g['avg_us']:.1f} | {g['tflops']:.1f} | {100 * g['frac']:.1f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out
