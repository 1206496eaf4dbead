"""Helpers for the measurement side: source fingerprint of the HIP kernels and
rocprofv3 counter summaries.

`counter_summary` turns the `*_counter_collection.csv` files of rocprofv3
`--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs into bytes per dispatch and
kernel, scaled by the readings of a plain device copy of known size (the
counters' unit differs from bytes on this device: FETCH_SIZE reads half of the
bytes a 128-byte-line copy moves).  The summary records the fingerprint of the
kernel sources it was taken with; `traffic_for` returns nothing once the
sources have changed.
"""
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

_HERE = os.path.dirname(os.path.abspath(__file__))


def source_fingerprint():
    """sha256 over the HIP sources and headers of the library."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")) + glob.glob(os.path.join(_HERE, "csrc", "*.hpp"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name):
    m = re.match(r"(?:void )?(?:bfgp::)?([A-Za-z_0-9]+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name


def _read(csv_path, counter):
    per = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        per[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in per.items()}


def counter_summary(fetch_csv, write_csv, copy_bytes, copy_kernel="__amd_rocclr_copyBuffer"):
    """{(kernel, grid): {fetch_bytes, write_bytes}} per dispatch, calibrated by
    the copy of `copy_bytes` bytes each way (the largest copy dispatch)."""
    fetch = _read(fetch_csv, "FETCH_SIZE")
    write = _read(write_csv, "WRITE_SIZE")
    cf = max((v for (k, g), v in fetch.items() if k == copy_kernel), default=None)
    cw = max((v for (k, g), v in write.items() if k == copy_kernel), default=None)
    if not cf or not cw:
        raise ValueError("no copy dispatch to calibrate against")
    sf, sw = copy_bytes / cf, copy_bytes / cw
    out = {}
    for key in fetch:
        if key[0] == copy_kernel:
            continue
        out[f"{key[0]}@{key[1]}"] = {"fetch_bytes": fetch[key] * sf, "write_bytes": write.get(key, 0.0) * sw}
    return {"fingerprint": source_fingerprint(), "fetch_scale_bytes_per_unit": sf, "write_scale_bytes_per_unit": sw,
            "per_dispatch": out}


# profiling stage name -> kernel instantiation name prefix in counter files
STAGE_KERNELS = {
    "k_vband_agg": "k_vband<64, true, false>", "k_vband_agg_big": "k_vband<64, true, true>",
    "k_vband": "k_vband<64, false, false>", "k_vband_big": "k_vband<64, false, true>",
    "k_hrow": "k_hrow<", "k_fir": "k_fir<", "k_bwd": "k_bwd<",
}


def traffic_for(summary_path, stage, grid):
    """Calibrated HBM bytes (fetch + write) per dispatch of the kernel behind
    profiling stage `stage` launched with `grid` threads, or None when absent
    or taken with other kernel sources."""
    try:
        s = json.load(open(summary_path))
    except (OSError, ValueError):
        return None
    if s.get("fingerprint") != source_fingerprint():
        return None
    want = STAGE_KERNELS.get(stage, stage)
    for key, v in s["per_dispatch"].items():
        name, g = key.rsplit("@", 1)
        if int(g) == grid and (name == want or name.startswith(want)):
            return v["fetch_bytes"] + v["write_bytes"]
    return None
