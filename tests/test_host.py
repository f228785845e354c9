"""Host-side checks that need no GPU: the benchmark's contract for more
than one GPU, the HBM-traffic arithmetic, and the seeded generators."""
import csv
import os
import subprocess
import sys

import numpy as np

from paper_2111_10980_amd import inputs, traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_is_scaled_by_the_copy_kernel(tmp_path):
    # the copy kernel moves 1 GiB each way; its counters read half (fetch) and
    # all (write) of that, so the kernel's readings scale by 2 and 1
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fetch, "FETCH_SIZE", [("k_copy(x)", 524288.0), ("void k_apply3(a)", 1000.0),
                                          ("void k_apply3(a)", 3000.0)])
    _write_counters(write, "WRITE_SIZE", [("k_copy(x)", 1048576.0), ("void k_apply3(a)", 500.0),
                                          ("void k_apply3(a)", 500.0)])
    t = traffic.traffic(str(fetch), str(write), "k_apply3")
    assert t["launches"] == 2
    assert abs(t["fetch_bytes_per_launch"] - 2000.0 * 2048.0) < 1e-6
    assert abs(t["write_bytes_per_launch"] - 500.0 * 1024.0) < 1e-6
    assert len(t["source_hash"]) == 16


def test_generators_are_deterministic_and_simple():
    for make in (lambda s: inputs.rmat(10, 8, s), lambda s: inputs.erdos_renyi(500, 2000, s),
                 lambda s: inputs.rmat_paper(9, 8, s),
                 lambda s: inputs.chung_lu_planted(2000, 8.0, 2.1, 3, 5, 9, s)):
        a, b, c = make(1), make(1), make(2)
        assert a.sha256() == b.sha256() and a.sha256() != c.sha256()
        rp, col = a.row_ptr, a.col
        for v in range(a.n):
            row = col[rp[v]:rp[v + 1]]
            assert (np.diff(row) > 0).all() and not (row == v).any()
        # symmetric
        src = np.repeat(np.arange(a.n), np.diff(rp))
        fwd = set(zip(src.tolist(), col.tolist()))
        assert all((y, x) in fwd for x, y in fwd)


def test_batch_and_serving_recipes():
    order = inputs.batch_order()
    assert sorted(order.tolist()) == list(range(4096))
    g = inputs.batch_graph(5)
    assert 50 <= g.n <= 5000
    jobs = inputs.serving_stream(100.0, 200, max_scale=12)
    t = [j.arrival_s for j in jobs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert all(10 <= j.scale <= 12 and 8 <= j.edge_factor <= 16 for j in jobs)
    assert all(1 <= j.r <= 3 and j.r + 1 <= j.s <= j.r + 2 for j in jobs)
    # the same job sequence at another rate, only the arrival times scale
    other = inputs.serving_stream(50.0, 200, max_scale=12)
    assert [(j.scale, j.r, j.s, j.graph_seed) for j in jobs] == \
        [(j.scale, j.r, j.s, j.graph_seed) for j in other]
