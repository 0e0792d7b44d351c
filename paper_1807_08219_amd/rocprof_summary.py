"""Text summaries of rocprofv3 CSV output (kernel statistics, HBM traffic).

  python -m paper_1807_08219_amd.rocprof_summary stats KERNEL_STATS_CSV
      one markdown table row per library kernel: calls, average and total time.

  python -m paper_1807_08219_amd.rocprof_summary traffic FETCH_CSV WRITE_CSV KERNEL COPY_BYTES
      HBM bytes per launch of KERNEL from two counter-collection runs (one
      with FETCH_SIZE, one with WRITE_SIZE, both in KiB per dispatch).  Each
      counter is scaled by what it reads for the largest plain device copy in
      the same run, of COPY_BYTES read and COPY_BYTES written, so that the
      result does not depend on how the counter aggregates over the memory
      channels.  Prints a JSON object.
"""
from __future__ import annotations

import collections
import csv
import json
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name[5:] if name.startswith("void ") else name


def kernel_table(stats_csv: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | avg us | total ms |", "|---|---:|---:|---:|"]
    for r in rows:
        if "ifem" not in r["Name"]:
            continue
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} |")
    return "\n".join(out)


def _per_dispatch(counter_csv: str, counter: str):
    """{kernel: [value per dispatch]} for one counter (rows of one dispatch summed)."""
    acc = collections.defaultdict(float)
    names = {}
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] != counter:
            continue
        d = r["Dispatch_Id"]
        acc[d] += float(r["Counter_Value"])
        names[d] = _short(r["Kernel_Name"])
    out = collections.defaultdict(list)
    for d, v in acc.items():
        out[names[d]].append(v)
    return out


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int) -> dict:
    rec = {"kernel": kernel, "copy_bytes": copy_bytes}
    total = 0.0
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        per = _per_dispatch(path, counter)
        copies = per.get(COPY_KERNEL, [])
        if not copies:
            raise SystemExit(f"no {COPY_KERNEL} dispatch in {path}")
        ref_kib = max(copies)
        scale = copy_bytes / (ref_kib * 1024.0)  # true bytes per counted byte
        vals = [v for name, lst in per.items() if name == kernel for v in lst]
        if not vals:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        kib = sum(vals) / len(vals)
        bytes_ = kib * 1024.0 * scale
        key = "fetch" if counter == "FETCH_SIZE" else "write"
        rec[f"{key}_kib_per_launch"] = round(kib, 1)
        rec[f"{key}_copy_kib"] = round(ref_kib, 1)
        rec[f"{key}_scale"] = round(scale, 4)
        rec[f"{key}_bytes_per_launch"] = int(bytes_)
        rec[f"{key}_launches"] = len(vals)
        total += bytes_
    rec["hbm_bytes_per_launch"] = int(total)
    return rec


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(kernel_table(argv[1]))
    elif len(argv) >= 5 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], int(argv[4])), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
