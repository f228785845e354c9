"""HBM traffic of a kernel from rocprofv3 counter CSVs.

Two ``rocprofv3 --pmc`` runs of the same command, one with FETCH_SIZE and one
with WRITE_SIZE (both in KiB per dispatch), are reduced to bytes per launch of
the kernel of interest.  Each counter is scaled by what it reads for the
plain copy kernel ``k_copy`` of the roofline probes, which moves a known
number of bytes (1 GiB read + 1 GiB written per dispatch), so the figure is in
true bytes whatever the counter's unit convention.

The result is written as JSON together with a hash of the HIP sources that
define the peel kernels (the peel module and the headers it includes), so a
reader can tell whether the numbers still describe the current kernels.

Usage:
  python -m paper_2111_10980_amd.traffic FETCH_CSV WRITE_CSV KERNEL_REGEX OUT_JSON
  python -m paper_2111_10980_amd.traffic --counters CSV [CSV ...] > table.md
The second form reduces any counter CSVs to one row per kernel: dispatches
and the mean value of every counter per dispatch.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30  # k_copy: bytes read (and written) per dispatch


KERNEL_SOURCES = ("nd_peel.hip", "nd_internal.h", "nd_host.h")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _per_kernel(path: str, counter: str, kernel_re: str):
    rows = list(csv.DictReader(open(path)))
    rx = re.compile(kernel_re)
    tot, n, copy_tot, copy_n = 0.0, 0, 0.0, 0
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        if rx.search(name):
            tot += v
            n += 1
        elif "k_copy" in name:
            copy_tot += v
            copy_n += 1
    return tot, n, copy_tot, copy_n


def traffic(fetch_csv: str, write_csv: str, kernel_re: str) -> dict:
    f, nf, cf, ncf = _per_kernel(fetch_csv, "FETCH_SIZE", kernel_re)
    w, nw, cw, ncw = _per_kernel(write_csv, "WRITE_SIZE", kernel_re)
    if not (nf and nw and ncf and ncw):
        raise SystemExit("kernel or copy calibration dispatches missing from the CSVs")
    fetch_scale = COPY_BYTES / (cf / ncf)
    write_scale = COPY_BYTES / (cw / ncw)
    fetch_b = f * fetch_scale / nf
    write_b = w * write_scale / nw
    return {
        "kernel_regex": kernel_re,
        "launches": nf,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": fetch_b + write_b,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "copy_fetch_kib_per_dispatch": cf / ncf,
        "copy_write_kib_per_dispatch": cw / ncw,
        "source_hash": source_hash(),
    }


def counter_table(paths) -> str:
    """Markdown table: per kernel, dispatches and each counter's mean per dispatch."""
    acc = {}
    names = []
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = re.sub(r"\(.*", "", r["Kernel_Name"].replace("(anonymous namespace)::", ""))
            k = k.replace("void ", "")
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            d = acc.setdefault(k, {})
            v = d.setdefault(c, [0.0, 0])
            v[0] += float(r["Counter_Value"])
            v[1] += 1
    lines = ["| kernel | dispatches | " + " | ".join(names) + " |",
             "|---|---:|" + "---:|" * len(names)]
    for k, d in sorted(acc.items()):
        n = max(v[1] for v in d.values())
        cells = []
        for c in names:
            v = d.get(c)
            cells.append(f"{v[0] / v[1]:.4g}" if v else "")
        lines.append(f"| {k} | {n} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "--counters":
        print(counter_table(sys.argv[2:]))
        sys.exit(0)
    if len(sys.argv) != 5:
        print(__doc__)
        sys.exit(2)
    out = traffic(sys.argv[1], sys.argv[2], sys.argv[3])
    with open(sys.argv[4], "w") as fh:
        json.dump(out, fh, indent=2)
    print(json.dumps(out, indent=2))
