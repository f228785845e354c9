"""Write the oracle's exact results for the full-size workloads -- TEST
INFRASTRUCTURE ONLY.

Runs the plain sequential CPU oracle (``oracle/nd_oracle.c``, one thread) on a
full-size seeded workload and stores, under ``tests/golden/``, what a GPU
decomposition of the same input must reproduce exactly (Algorithm 2 returns
the nucleus number of every r-clique; the round structure follows from the
bucket loop):

- the input's SHA-256 (so a changed generator is caught before any compare);
- n_r, n_s, the number of rounds rho, the maximum nucleus number;
- every round's size |A_t| and level k (lists, and SHA-256 of their uint32
  little-endian bytes);
- SHA-256 of the canonical output: the r-clique rows (int32 little-endian,
  each row's original ids ascending, rows in lexicographic order), the initial
  counts and the nucleus numbers (uint32 little-endian, in row order);
- the histogram of nucleus numbers, the total of decrements;
- the oracle's wall time for one decomposition (validation, r-clique table,
  count and peel; the Python copy-out excluded), the host's logical CPU count
  and CPU model, and the one thread the oracle uses.

Only ``oracle/`` and the seeded generators are imported; nothing here touches
the GPU library.

    python oracle/fullsize_golden.py rmat18_34
    python oracle/fullsize_golden.py chunglu1m_45
    python oracle/fullsize_golden.py chunglu1m_24
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
# run as a script, the oracle folder itself would shadow the package name
sys.path[:] = [p for p in sys.path if os.path.abspath(p or ".") != _HERE]
sys.path.insert(0, _ROOT)

from oracle import oracle  # noqa: E402
from paper_2111_10980_amd import inputs  # noqa: E402

GOLDEN_DIR = os.path.join(_ROOT, "tests", "golden")

# name -> (recipe text, graph factory, r, s)
WORKLOADS = {
    "rmat18_34": ("rMAT scale 18, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 18",
                  inputs.rmat18, 3, 4),
    "chunglu1m_45": ("Chung-Lu n=1e6, average degree 20, exponent 2.1, 200 planted cliques "
                     "of 20-60 vertices, seed 2021", inputs.chung_lu_1m, 4, 5),
    "chunglu1m_24": ("Chung-Lu n=1e6, average degree 20, exponent 2.1, 200 planted cliques "
                     "of 20-60 vertices, seed 2021", inputs.chung_lu_1m, 2, 4),
}


def sha_u32(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def sha_i32(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, check=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.CalledProcessError):
        pass
    return platform.processor() or "unknown"


def path_for(name: str) -> str:
    return os.path.join(GOLDEN_DIR, f"fullsize_{name}.json")


def run(name: str) -> dict:
    recipe, factory, r, s = WORKLOADS[name]
    g = factory()
    print(f"[golden] {name}: n={g.n} m={g.m} r={r} s={s}; oracle running", flush=True)
    t0 = time.perf_counter()
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    wall = time.perf_counter() - t0
    if res.counts.size and int(res.counts.max()) > 0xFFFFFFFF:
        raise SystemExit("a count exceeds 32 bits")
    kappa = res.kappa.astype(np.uint32)
    hist_k, hist_n = np.unique(kappa, return_counts=True)
    rec = {
        "workload": name,
        "recipe": recipe,
        "r": r,
        "s": s,
        "input_sha256": g.sha256(),
        "n": g.n,
        "m": g.m,
        "n_r": res.n_r,
        "n_s": res.n_s,
        "rounds": res.rounds,
        "max_kappa": res.max_kappa,
        "decrements": res.decrements,
        "round_sizes": [int(x) for x in res.round_sizes],
        "round_k": [int(x) for x in res.round_k],
        "round_sizes_sha256": sha_u32(res.round_sizes),
        "round_k_sha256": sha_u32(res.round_k),
        "rows_sha256": sha_i32(res.rcliques),
        "counts_sha256": sha_u32(res.counts),
        "kappa_sha256": sha_u32(kappa),
        "kappa_hist": [[int(k), int(c)] for k, c in zip(hist_k, hist_n)],
        "digest_format": "rows int32 LE (ids ascending per row, rows lexicographic); counts, "
                         "kappa, round sizes and levels uint32 LE",
        "oracle_wall_s": round(wall, 3),
        "oracle_threads": 1,
        "host_nproc": os.cpu_count(),
        "host_cpu": cpu_model(),
        "script": "python oracle/fullsize_golden.py " + name,
    }
    return rec


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(WORKLOADS))
    args = ap.parse_args()
    rec = run(args.name)
    os.makedirs(GOLDEN_DIR, exist_ok=True)
    tmp = path_for(args.name) + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    os.replace(tmp, path_for(args.name))
    print(f"[golden] {args.name}: n_r={rec['n_r']} n_s={rec['n_s']} rounds={rec['rounds']} "
          f"max kappa={rec['max_kappa']} in {rec['oracle_wall_s']} s", flush=True)


if __name__ == "__main__":
    main()
