"""Summaries of rocprofv3 counter runs.

`python -m paper_2511_23438_amd.profiling counters <csv> <kernel-substring>
<calibration-kernel-substring> <calibration-bytes> <counter>` reads a
`*_counter_collection.csv` written by `rocprofv3 --pmc <counter>` and prints
the mean counter value per dispatch of the named kernel, scaled by the ratio
between the known size of a plain copy (the calibration dispatch) and what
the same counter read for it.
"""
from __future__ import annotations

import csv
import json
import sys


def per_dispatch(path: str, counter: str) -> list[tuple[str, float]]:
    """(kernel name, counter value) per dispatch, summing counter instances."""
    acc: dict[str, list] = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            key = row.get("Dispatch_Id") or row.get("Correlation_Id")
            name = row.get("Kernel_Name", "")
            val = float(row.get("Counter_Value", 0.0))
            if key not in acc:
                acc[key] = [name, 0.0]
            acc[key][1] += val
    return [(v[0], v[1]) for v in acc.values()]


def summarise(path: str, kernel: str, calib_kernel: str, calib_bytes: float,
              counter: str) -> dict:
    rows = per_dispatch(path, counter)
    cal = [v for (n, v) in rows if calib_kernel in n]
    ker = [v for (n, v) in rows if kernel in n]
    if not cal or not ker:
        raise SystemExit("kernel or calibration dispatch not found")
    # counters report KiB; the calibration copy reads and writes calib_bytes
    cal_kib = max(cal)
    scale = (calib_bytes / 1024.0) / cal_kib if cal_kib > 0 else float("nan")
    mean_kib = sum(ker) / len(ker)
    return {"counter": counter, "kernel": kernel, "dispatches": len(ker),
            "mean_kib_per_dispatch": mean_kib, "calibration_kib": cal_kib,
            "calibration_bytes": calib_bytes, "scale": scale,
            "bytes_per_dispatch": mean_kib * 1024.0 * scale}


if __name__ == "__main__":
    if len(sys.argv) == 7 and sys.argv[1] == "counters":
        print(json.dumps(summarise(sys.argv[2], sys.argv[3], sys.argv[4],
                                   float(sys.argv[5]), sys.argv[6])))
    else:
        print(__doc__)
        sys.exit(2)
