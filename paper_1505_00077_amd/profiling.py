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


def _code_only(text):
    """C++ source with comments removed and whitespace collapsed (string
    literals kept), so that edits to comments leave the fingerprint alone."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_fingerprint():
    """sha256 over the code (comments and whitespace aside) of the library's
    HIP sources and headers."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")) + glob.glob(os.path.join(_HERE, "csrc", "*.hpp"))):
        h.update(os.path.basename(path).encode())
        with open(path, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
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


def traffic_for(summary_path, launches):
    """Mean calibrated HBM bytes (fetch + write) per dispatch over `launches`,
    a list of (kernel instantiation name as in the counter files, grid size in
    threads); None when any of them is absent or the summary was taken with
    other kernel sources."""
    try:
        with open(summary_path) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("fingerprint") != source_fingerprint() or not launches:
        return None
    vals = []
    for name, grid in launches:
        v = s["per_dispatch"].get(f"{name}@{int(grid)}")
        if v is None:
            return None
        vals.append(v["fetch_bytes"] + v["write_bytes"])
    return sum(vals) / len(vals)


def kernel_stats_table(stats_csv, top=12):
    """Markdown table of a rocprofv3 `--stats` kernel summary (name, calls,
    average and total duration), the `top` kernels by total time."""
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | total us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    return "\n".join(out)


def kernel_trace_table(trace_csv, top=16):
    """Markdown table of a rocprofv3 `--kernel-trace` CSV grouped by kernel
    and grid size (calls, average and total duration), by total time."""
    per = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        per[(_short(r["Kernel_Name"]), grid)].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in per.values())
    rows = sorted(per.items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | grid | calls | avg us | total us | share |", "|---|---:|---:|---:|---:|---:|"]
    for (name, grid), v in rows[:top]:
        out.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / len(v):.2f} | {sum(v):.1f} | "
                   f"{100 * sum(v) / total:.1f}% |")
    return "\n".join(out)


def sq_table(counter_csv, kernels=None):
    """Markdown table of SQ counters per dispatch (mean over the dispatches of
    each kernel and grid size) from a rocprofv3 `--pmc SQ_...` run: wave64
    VALU, LDS and SALU instructions, waves, and the shader engines' busy
    cycles (summed over the engines)."""
    per = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(counter_csv)):
        per[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["| kernel | grid | dispatches | VALU instr | LDS instr | SALU instr | waves | busy cycles |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    rows = []
    for (name, grid), c in per.items():
        if kernels and not any(name.startswith(k) for k in kernels):
            continue
        m = {k: sum(v) / len(v) for k, v in c.items()}
        n = max(len(v) for v in c.values())
        rows.append((-m.get("SQ_INSTS_VALU", 0), f"| `{name}` | {grid} | {n} | {m.get('SQ_INSTS_VALU', 0):.4g} | "
                     f"{m.get('SQ_INSTS_LDS', 0):.4g} | {m.get('SQ_INSTS_SALU', 0):.4g} | "
                     f"{m.get('SQ_WAVES', 0):.4g} | {m.get('SQ_BUSY_CYCLES', 0):.4g} |"))
    out += [r for _, r in sorted(rows)]
    return "\n".join(out)


def main(argv):
    """python -m paper_1505_00077_amd.profiling counters FETCH.csv WRITE.csv COPY_BYTES
       python -m paper_1505_00077_amd.profiling stats KERNEL_STATS.csv
       python -m paper_1505_00077_amd.profiling trace KERNEL_TRACE.csv
       python -m paper_1505_00077_amd.profiling sq SQ_COUNTERS.csv [kernel prefix ...]"""
    if len(argv) >= 4 and argv[0] == "counters":
        print(json.dumps(counter_summary(argv[1], argv[2], int(argv[3])), indent=1))
    elif len(argv) >= 2 and argv[0] == "stats":
        print(kernel_stats_table(argv[1]))
    elif len(argv) >= 2 and argv[0] == "trace":
        print(kernel_trace_table(argv[1]))
    elif len(argv) >= 2 and argv[0] == "sq":
        print(sq_table(argv[1], argv[2:] or None))
    else:
        print(main.__doc__)
        return 2
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main(sys.argv[1:]))
