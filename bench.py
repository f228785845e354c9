#!/usr/bin/env python3
"""Benchmark: (3,4) nucleus decomposition of an rMAT scale-18 graph on one GPU.

One step = the whole hot path on a graph already resident in HBM:
validation, orientation + relabeling, r-clique table build, s-clique
counting, bucketed peeling and emission of (r-clique rows, kappa), through
the C ABI.  The metric is whole-job s-clique peel updates per second: every
s-clique is destroyed exactly once while peeling, so one step performs n_s
updates and value = n_s / (seconds per step).

Prints ONE JSON line.  Besides the driver's fields it carries
  roofline      the dominant kernel's algorithmic HBM bytes / its measured
                time (HIP events on the library's stream over the timed
                steps) against the MI355X HBM peak, plus the access-pattern
                roofline T_roof = max(stream bytes / copy rate, probes /
                random-gather rate, atomics / random-atomic rate) with the
                three ceilings measured in the same run;
  cpu_baseline  the CPU oracle (single thread) timed in this run on a bounded
                sample of the same graph family (rMAT scale 12, same a..d),
                with the host's core count and CPU model; next to it the
                oracle's stored run on the full input itself (same SHA-256)
                from tests/golden/, with the host it ran on.
"""
import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
SLOT_BYTES = 16                # one r-clique table slot {key, count, stamp}

BATCH_WORKLOAD = "batch4096_34"
SERVE_WORKLOAD = "serve_rmat"
SERVE_CLASSES_WORKLOAD = "serve_classes"
SWEEP_WORKLOAD = "rmat_density_sweep"

WORKLOADS = {
    # name: (generator, r, s, description)
    "rmat18_34": ("rmat18", 3, 4, "rMAT scale 18, edge factor 16, a=.57 b=.19 c=.19 d=.05, "
                  "symmetrised, loops/duplicates removed; (3,4) nucleus"),
    "er2000_23": ("er_2000", 2, 3, "Erdos-Renyi G(n=2000, m=10000); (2,3) nucleus"),
    "rmat18_23": ("rmat18", 2, 3, "rMAT scale 18, edge factor 16, a=.57 b=.19 c=.19 d=.05, "
                  "symmetrised, loops/duplicates removed; (2,3) nucleus (k-truss)"),
    "chunglu1m_45": ("chung_lu_1m", 4, 5, "Chung-Lu n=1e6, avg degree 20, exponent 2.1, "
                     "200 planted cliques of size 20-60; (4,5) nucleus"),
    "chunglu1m_24": ("chung_lu_1m", 2, 4, "Chung-Lu n=1e6, avg degree 20, exponent 2.1, "
                     "200 planted cliques of size 20-60; (2,4) nucleus"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, check=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, ValueError, RuntimeError):
        pass
    return "unknown"


def full_oracle_run(workload, input_sha):
    """The oracle's stored run on the full input (tests/golden/), if it is
    the same input."""
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("input_sha256") != input_sha:
        return None
    return {"value": rec["n_s"] / rec["oracle_wall_s"], "unit": "s-clique peel updates/s",
            "cores": rec["oracle_threads"], "kind": "oracle", "wall_s": rec["oracle_wall_s"],
            "input_sha256": input_sha, "host_cpu": rec["host_cpu"],
            "host_nproc": rec["host_nproc"],
            "sample": f"the whole {workload} input (n_s={rec['n_s']}), validation + table + "
                      f"count + peel, one thread, stored by {rec['script']}"}


def cpu_baseline(r, s, scale=12, seed=18):
    """The oracle as it stands, single-threaded, on rMAT scale `scale`."""
    from oracle import oracle
    from paper_2111_10980_amd import inputs
    g = inputs.rmat(scale, 16, seed)
    t0 = time.perf_counter()
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    dt = time.perf_counter() - t0
    return {"value": res.n_s / dt, "unit": "s-clique peel updates/s", "cores": 1,
            "kind": "oracle", "host_cpu": host_cpu(), "host_nproc": os.cpu_count(),
            "sample": f"rMAT scale {scale} edge factor 16 (same a..d, seed {seed}; n={g.n}, "
                      f"m={g.m}, n_s={res.n_s}), ({r},{s}), validation + table + count + peel, "
                      f"{dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18_34",
                    choices=sorted(WORKLOADS) + [BATCH_WORKLOAD, SERVE_WORKLOAD, SWEEP_WORKLOAD,
                                                 SERVE_CLASSES_WORKLOAD])
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--rates", default="5,10,20,40",
                    help="serving: Poisson arrival rates (jobs/s) to sweep")
    ap.add_argument("--serve-jobs", type=int, default=300, help="serving: measured jobs per rate")
    ap.add_argument("--serve-warmup", type=int, default=30, help="serving: warm-up jobs per rate")
    ap.add_argument("--max-scale", type=int, default=11, help="serving: largest rMAT scale")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--classes", default="",
                    help="serving classes: only these (r,s), e.g. '3,4;3,5' (default all)")
    ap.add_argument("--class-cap-s", type=float, default=20.0,
                    help="serving classes: skip a class at the next scale once one job of it "
                         "would take longer than this")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--orient", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--contract", action="store_true",
                    help="(2,3): graph contraction on (for the before/after comparison)")
    ap.add_argument("--levels", type=int, default=0, choices=[0, 2, 3],
                    help="r-clique table levels (3: three-level table, r >= 4)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: default schedules instead of the autotuner's choice")
    ap.add_argument("--tune-sample", type=int, default=256,
                    help="batched: graphs in the autotuner's held-out sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2111_10980_amd as nd
    from paper_2111_10980_amd import inputs

    if args.workload == BATCH_WORKLOAD:
        return bench_batch(args)
    if args.workload == SERVE_WORKLOAD:
        return bench_serve(args)
    if args.workload == SERVE_CLASSES_WORKLOAD:
        return bench_serve_classes(args)
    if args.workload == SWEEP_WORKLOAD:
        return bench_sweep(args)
    gen, r, s, desc = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = getattr(inputs, gen)() if args.seed is None else getattr(inputs, gen)(args.seed)
    log(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp, col = nd.to_device(g, dev)
    torch.cuda.synchronize()

    def step():
        return nd.decompose(rp, col, r, s, orient=args.orient, timing=True,
                            contract=args.contract, levels=args.levels)

    for i in range(args.warmup):
        d = step()
        log(f"[bench] warmup {i}: total {d.stats['ms']['total']:.1f} ms, rounds "
            f"{d.stats['rounds']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / max(1, args.steps)
    st = runs[-1].stats
    for d in runs:
        assert d.stats["n_s"] == st["n_s"] and d.stats["rounds"] == st["rounds"]
    n_s = st["n_s"]
    value = n_s / (ms_per_step / 1000.0)
    log(f"[bench] {args.steps} steps, {ms_per_step:.1f} ms/step; n_r={st['n_r']} n_s={n_s} "
        f"rounds={st['rounds']} max_kappa={st['max_kappa']} phases={st['ms']}")

    # ---- roofline of the dominant kernel, from the timed steps
    cnt_ms = sum(d.stats["count_kernel_ms"] for d in runs)
    peel_ms = sum(d.stats["peel_kernel_ms"] for d in runs)
    peel_launches = sum(d.stats["peel_launches"] for d in runs)
    c = comb(s, r)
    count_bytes = SLOT_BYTES * c * n_s * len(runs)
    peel_bytes = SLOT_BYTES * (c - 1) * n_s * len(runs)
    # the kernels the library times with HIP events on its own stream:
    # s = r+1 (r >= 2) peels through k_apply and counts directly; s >= r+2
    # peels through k_gen_apply and counts by listing; (1,2) uses k_peel
    if s == r + 1 and r >= 2:
        peel_name = "k_apply3" if r == 3 else f"k_apply<{r}>"
        count_name = "k_count_direct<2>" if r == 2 else f"k_count_group<{r}>"
    else:
        peel_name = f"k_gen_apply<{r}, {s}>" if s >= r + 2 else f"k_peel<{r}, {s}>"
        count_name = f"k_list_bitmap<{s}, W, CountOp<{r}, {s}>>"
    if peel_ms >= cnt_ms:
        kern, t_ms, nbytes, launches = peel_name, peel_ms, peel_bytes, peel_launches
    else:
        kern, t_ms, nbytes, launches = count_name, cnt_ms, count_bytes, len(runs)
    launches = max(1, launches)
    achieved = nbytes / (t_ms / 1000.0) / 1e9 if t_ms > 0 else 0.0
    n_launch = max(1, launches)
    # measured device ceilings over buffers the size of the r-clique table
    # (probes and decrements both land in its slots); k_copy inside also
    # calibrates the HBM counters
    table_bytes = st["table_slots"] * SLOT_BYTES
    ceil = nd.nd_roofline_measure(table_bytes, table_bytes)
    log(f"[bench] ceilings: {ceil}")
    # random-access model of the peel's update pass: every discovered s-clique
    # probes its C(s,r)-1 other slots; every decrement of a count still above
    # the level is a returning atomic
    probes = st["discoveries"] * (c - 1)
    t_probe = probes / (ceil["gather16_gops"] * 1e9)
    t_atom = st["atomics"] / (ceil["atomic_ret_gops"] * 1e9)
    t_stream = (nbytes / n_launch) * (launches / len(runs)) / (ceil["copy_gbs"] * 1e9)
    # the access-pattern roofline: the slowest of the three ceilings bounds
    # the pass; the serial figure adds probes and atomics (no overlap)
    roof_ms = 1000.0 * max(t_stream, t_probe, t_atom)
    model_ms = 1000.0 * (t_probe + t_atom)
    peel_step_ms = peel_ms / len(runs)
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kern.split('<')[0]}_{args.workload}.json")
    if os.path.exists(tfile):
        from paper_2111_10980_amd import traffic as tr
        rec = json.load(open(tfile))
        if rec.get("source_hash") == tr.source_hash():
            traffic = rec["traffic_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": kern, "launches_per_step": launches // max(1, len(runs)),
                "kernel_ms_per_step": round(t_ms / len(runs), 3),
                "algorithmic_bytes_per_launch": nbytes // n_launch,
                "count_kernel_ms_per_step": round(cnt_ms / len(runs), 3),
                "peel_kernel_ms_per_step": round(peel_ms / len(runs), 3),
                "measured_ceilings": {k: round(v, 3) for k, v in ceil.items()},
                "access_roofline": {
                    "formula": "T_roof = max(stream bytes / copy rate, probes / gather rate, "
                               "atomics / atomic rate); frac = T_roof / T_measured",
                    "probes": probes, "atomics": st["atomics"],
                    "t_stream_ms": round(1000.0 * t_stream, 3),
                    "t_probe_ms": round(1000.0 * t_probe, 3),
                    "t_atomic_ms": round(1000.0 * t_atom, 3),
                    "t_roof_ms": round(roof_ms, 3),
                    "measured_ms": round(peel_step_ms, 3),
                    "frac": round(roof_ms / peel_step_ms, 4) if peel_step_ms > 0 else None,
                    "serial_model_ms": round(model_ms, 2),
                    "serial_model_frac": round(model_ms / peel_step_ms, 4)
                    if peel_step_ms > 0 else None}}

    base = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on the bounded sample")
        base = cpu_baseline(r, s)
        log(f"[bench] cpu baseline: {base['value']:.4g} {base['unit']} ({base['sample']})")
        base["full_input"] = full_oracle_run(args.workload, g.sha256())

    out = {
        "metric": "s-clique peel updates/sec",
        "value": value,
        "unit": "s-cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "r": r, "s": s, "n": g.n,
                   "m": g.m, "n_r": st["n_r"], "n_s": n_s, "rounds": st["rounds"],
                   "max_kappa": st["max_kappa"], "orientation": ["degree", "core"][args.orient],
                   "max_out_degree": st["max_out_degree"], "decrements": st["decrements"],
                   "atomics": st["atomics"], "discoveries": st["discoveries"], "k_advances": st["k_advances"],
                   "table_slots": st["table_slots"], "contractions": st["contractions"],
                   "contract": bool(args.contract), "table_levels": args.levels or 2,
                   "key_words": st["key_words"], "phase_ms": st["ms"]},
        "roofline": roofline,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched (3,4) decomposition of many small uneven graphs in one fused
    run, against the same graphs decomposed one at a time (graphs/s)."""
    import numpy as np
    import torch
    import paper_2111_10980_amd as nd
    from paper_2111_10980_amd import inputs
    r, s = 3, 4
    count = args.batch_count
    t0 = time.perf_counter()
    order = inputs.batch_order(count) if count == 4096 else np.arange(count)
    # generated in worker processes before this process touches the GPU
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        gs = pool.map(inputs.batch_graph, [int(i) for i in order], chunksize=32)
    log(f"[bench] generated {count} graphs in {time.perf_counter() - t0:.1f}s: "
        f"sum n={sum(g.n for g in gs)}, sum m={sum(g.m for g in gs)}")
    torch.cuda.set_device(0)
    dev = [nd.to_device(g, "cuda:0") for g in gs]
    torch.cuda.synchronize()
    # schedules: the autotuner times each candidate on a held-out sample
    tune = None
    opts = {}
    if not args.no_autotune:
        t0 = time.perf_counter()
        best, rep = nd.nd_batch_autotune(dev, r, s, sample_count=args.tune_sample)
        opts = {"orient": best["orient"], "queue_depth": best["queue_depth"],
                "graph_rounds": bool(best["graph_rounds"])}
        tune = {"sample_graphs": rep["sample_graphs"], "chosen": opts,
                "seconds": round(time.perf_counter() - t0, 2),
                "candidates": [{k: c[k] for k in ("orient", "queue_depth", "graph_rounds", "ms")}
                               for c in rep["candidates"]]}
        log(f"[bench] autotune: {tune}")
    for _ in range(args.warmup):
        res = nd.decompose_batch(dev, r, s, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = nd.decompose_batch(dev, r, s, **opts)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / max(1, args.steps)
    st = res.stats
    log(f"[bench] batched: {batched_s * 1000:.1f} ms per batch, rounds {st['rounds']}, "
        f"n_r {st['n_r']}, n_s {st['n_s']}")
    # the same graphs, one decomposition (plan, run, destroy) after another,
    # with the same schedule options
    nd.decompose(*dev[0], r, s, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = []
    for i, (rp, col) in enumerate(dev):
        d = nd.decompose(rp, col, r, s, **opts)
        if i % 257 == 0:
            singles.append((i, d))
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - t0
    log(f"[bench] serial: {serial_s * 1000:.1f} ms for {count} graphs")
    # spot check: batched rows of sampled graphs equal their single runs
    rcl = res.rcliques.cpu().numpy()
    kap = res.kappa.cpu().numpy()
    for i, d in singles:
        a, b = int(res.row_offsets[i]), int(res.row_offsets[i + 1])
        x, y = rcl[a:b], d.rcliques.cpu().numpy()
        ox, oy = np.lexsort(x.T[::-1]), np.lexsort(y.T[::-1])
        assert np.array_equal(x[ox], y[oy]) and np.array_equal(kap[a:b][ox],
                                                               d.kappa.cpu().numpy()[oy])
    out = {
        "metric": "batched graphs/sec",
        "value": count / batched_s,
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched_s * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "serial_graphs_per_s": count / serial_s,
        "speedup_vs_serial": serial_s / batched_s,
        "autotune": tune,
        "config": {"workload": BATCH_WORKLOAD, "graphs": count, "r": r, "s": s,
                   "sum_n": int(sum(g.n for g in gs)), "sum_m": int(sum(g.m for g in gs)),
                   "n_r": st["n_r"], "n_s": st["n_s"], "rounds": st["rounds"],
                   "phase_ms": st["ms"]},
    }
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """The paper's rMAT density sweep (a=.5, b=c=.1, d=.3): scale 16, edge
    factor 4..32, for (2,3), (3,4) and (4,5); one timed decomposition per
    point after a warm-up, s-clique peel updates/s per point."""
    import torch
    import paper_2111_10980_amd as nd
    from paper_2111_10980_amd import inputs
    torch.cuda.set_device(0)
    points = []
    tot_ns, tot_s = 0, 0.0
    for ef in inputs.DENSITY_SWEEP_EF:
        g = inputs.rmat_paper(inputs.DENSITY_SWEEP_SCALE, ef, 5000 + ef)
        rp, col = nd.to_device(g, "cuda:0")
        for r, s in inputs.DENSITY_SWEEP_RS:
            for _ in range(args.warmup):
                nd.decompose(rp, col, r, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                d = nd.decompose(rp, col, r, s)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / max(1, args.steps)
            st = d.stats
            tot_ns += st["n_s"]
            tot_s += dt
            points.append({"edge_factor": ef, "m": g.m, "r": r, "s": s, "n_r": st["n_r"],
                           "n_s": st["n_s"], "rounds": st["rounds"], "max_kappa": st["max_kappa"],
                           "ms": dt * 1000.0, "s_cliques_per_s": st["n_s"] / dt})
            log(f"[bench] ef {ef:2d} ({r},{s}): m={g.m} n_r={st['n_r']} n_s={st['n_s']} "
                f"rounds={st['rounds']} {dt * 1000:.1f} ms")
    out = {
        "metric": "s-clique peel updates/sec",
        "value": tot_ns / tot_s,
        "unit": "s-cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tot_s * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": SWEEP_WORKLOAD, "scale": inputs.DENSITY_SWEEP_SCALE,
                   "abcd": [0.5, 0.1, 0.1, 0.3], "points": points},
    }
    print(json.dumps(out), flush=True)


def _serve_graph(job):
    from paper_2111_10980_amd import inputs
    return inputs.rmat(job.scale, job.edge_factor, job.graph_seed)


def _replay(nd, jobs, dev, workers, budget):
    """Submit each job at its arrival time; per job (latency ms, completion s,
    stats).  Latency = queueing + service, both timed inside the library."""
    import threading
    out = [None] * len(jobs)
    ids = [None] * len(jobs)
    submitted = threading.Semaphore(0)
    sv = nd.Server(workers, budget)

    def collect():
        for i in range(len(jobs)):
            submitted.acquire()
            j = ids[i]
            nd.nd_server_wait(sv.handle, j, -1)
            _, _, st, qms, sms = nd.nd_server_result(sv.handle, j, jobs[i].r, copy=False)
            nd.nd_server_release(sv.handle, j)
            out[i] = (qms + sms, st, sms)
            if (i + 1) % 100 == 0:
                log(f"[bench]   {i + 1}/{len(jobs)} jobs done ({workers} workers)")

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    sub_t = [0.0] * len(jobs)
    for i, jb in enumerate(jobs):
        wait = t0 + jb.arrival_s - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        sub_t[i] = time.perf_counter() - t0
        ids[i] = nd.nd_server_submit(sv.handle, *dev[i], jb.r, jb.s)
        submitted.release()
    th.join()
    sv.close()
    return [(lat, sub_t[i] + lat / 1000.0, st, sms) for i, (lat, st, sms) in enumerate(out)]


def bench_serve(args):
    """Poisson stream of (rMAT graph, r, s) jobs replayed against the server:
    continuous batching (several worker streams) against one job at a time,
    at the same arrival times; p50/p99 latency and completed jobs/s."""
    import numpy as np
    import torch
    import paper_2111_10980_amd as nd
    from paper_2111_10980_amd import inputs
    rates = [float(x) for x in args.rates.split(",")]
    total = args.serve_warmup + args.serve_jobs
    base = inputs.serving_stream(1.0, total, seed=7, min_scale=10, max_scale=args.max_scale)
    t0 = time.perf_counter()
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        gs = pool.map(_serve_graph, base, chunksize=16)
    log(f"[bench] generated {total} serving graphs in {time.perf_counter() - t0:.1f}s "
        f"(scales 10..{args.max_scale}), sum m={sum(g.m for g in gs)}")
    torch.cuda.set_device(0)
    dev = [nd.to_device(g, "cuda:0") for g in gs]
    torch.cuda.synchronize()
    budget = int(args.hbm_budget_gb * (1 << 30))
    # warm the library (kernels loaded, pool grown) outside the measurement
    d = nd.decompose(*dev[0], base[0].r, base[0].s)
    torch.cuda.synchronize()
    sweep = []
    ref_stats = None
    for lam in rates:
        jobs = [inputs.Job(j.arrival_s / lam, j.scale, j.edge_factor, j.r, j.s, j.graph_seed)
                for j in base]
        row = {"rate": lam}
        for mode, workers in (("continuous", args.serve_workers), ("one_at_a_time", 1)):
            res = _replay(nd, jobs, dev, workers, budget)
            meas = res[args.serve_warmup:]
            lat = np.array([x[0] for x in meas])
            start = jobs[args.serve_warmup].arrival_s
            end = max(x[1] for x in meas)
            stats = [(x[2]["n_r"], x[2]["n_s"], x[2]["max_kappa"]) for x in res]
            if ref_stats is None:
                ref_stats = stats
            if mode == "one_at_a_time" and lam == rates[0]:
                per = {}
                for jb, x in zip(jobs, res):
                    per.setdefault((jb.scale, jb.r, jb.s), []).append(x[3])
                log("[bench] service ms by (scale,r,s), one at a time: " + ", ".join(
                    f"{k}:{np.mean(v):.1f}x{len(v)}" for k, v in sorted(per.items())))
            # the same jobs give the same results whatever the mode and rate
            assert stats == ref_stats, "served results differ between runs"
            row[mode] = {"workers": workers, "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)),
                         "mean_ms": float(lat.mean()),
                         "jobs_per_s": len(meas) / max(end - start, 1e-9)}
            log(f"[bench] rate {lam:g}/s {mode:14s} p50 {row[mode]['p50_ms']:8.1f} ms  "
                f"p99 {row[mode]['p99_ms']:8.1f} ms  {row[mode]['jobs_per_s']:7.1f} jobs/s")
        sweep.append(row)
    # headline: the highest rate at which continuous batching keeps up with
    # the arrivals (completed rate >= 90% of offered), else the lowest rate
    ok = [r_ for r_ in sweep if r_["continuous"]["jobs_per_s"] >= 0.9 * r_["rate"]]
    head = ok[-1] if ok else sweep[0]
    c = head["continuous"]
    classes = {}
    for jb in base:
        classes.setdefault(f"s{jb.scale}", 0)
        classes[f"s{jb.scale}"] += 1
    out = {
        "metric": "serving throughput at p50/p99 latency",
        "value": c["jobs_per_s"],
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": args.serve_jobs,
        "warmup": args.serve_warmup,
        "ms_per_step": 1000.0 / c["jobs_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "p50_ms": c["p50_ms"],
        "p99_ms": c["p99_ms"],
        "config": {"workload": SERVE_WORKLOAD, "rate": head["rate"],
                   "jobs": args.serve_jobs, "warmup_jobs": args.serve_warmup,
                   "scales": [10, args.max_scale], "edge_factor": [8, 16], "r": [1, 3],
                   "s": "r+1..r+2", "hbm_budget_gb": args.hbm_budget_gb,
                   "workers": args.serve_workers, "sweep": sweep},
    }
    print(json.dumps(out), flush=True)


def bench_serve_classes(args):
    """Service time of every job class of the serving mix (rMAT, r in 1..3,
    s in r+1..r+2) alone on the GPU, scale 10 up to 20, at edge factor 16 (the
    heaviest of the mix's 8..16), one warm-up and one timed decomposition per
    point.  A class stops growing in scale once its next job would take longer
    than --class-cap-s (estimated from the growth of the last two scales).  The
    mix's mean service time over scale ~U{10..20} and (r,s) ~U then bounds the
    arrival rate one GPU sustains; classes not measured are reported, and the
    bound is given over the measured scales only."""
    import numpy as np
    import torch
    import paper_2111_10980_amd as nd
    from paper_2111_10980_amd import inputs
    torch.cuda.set_device(0)
    classes = [(r, s) for r in (1, 2, 3) for s in (r + 1, r + 2)]
    only = [tuple(int(x) for x in c.split(",")) for c in args.classes.split(";")] \
        if args.classes else classes
    table = {}
    failed = {}
    for r, s in classes:
        if (r, s) not in only:
            continue
        prev = []
        for scale in range(10, 21):
            if len(prev) >= 2:
                growth = prev[-1] / max(prev[-2], 1e-3)
                if prev[-1] * growth > args.class_cap_s:
                    log(f"[bench] ({r},{s}) stops before scale {scale}: next job ~"
                        f"{prev[-1] * growth:.1f} s")
                    break
            g = inputs.rmat(scale, 16, 7000 + scale)
            rp, col = nd.to_device(g, "cuda:0")
            try:
                nd.decompose(rp, col, r, s)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d = nd.decompose(rp, col, r, s)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            except (torch.OutOfMemoryError, nd.NdError) as e:  # does not fit one GPU
                failed[f"({r},{s}) s{scale}"] = str(e)[:160]
                log(f"[bench] ({r},{s}) scale {scale}: {str(e)[:160]}")
                del rp, col
                nd.nd_release_cached()
                torch.cuda.empty_cache()
                break
            prev.append(dt)
            table[(r, s, scale)] = {"ms": round(1000 * dt, 2), "n_r": d.stats["n_r"],
                                    "n_s": d.stats["n_s"], "rounds": d.stats["rounds"]}
            log(f"[bench] ({r},{s}) scale {scale}: {1000 * dt:.1f} ms, n_r {d.stats['n_r']}, "
                f"n_s {d.stats['n_s']}")
            del rp, col, d
            nd.nd_release_cached()
            torch.cuda.empty_cache()
    measured_scales = sorted({k[2] for k in table})
    full = [sc for sc in measured_scales if all((r, s, sc) in table for r, s in only)]
    top = max(full) if full else 10
    mean_ms = float(np.mean([table[(r, s, sc)]["ms"] for r, s in only
                             for sc in range(10, top + 1)])) if full else float("nan")
    out = {
        "metric": "serving: sustainable arrival rate of one GPU (mean service time bound)",
        "value": 1000.0 / mean_ms,
        "unit": "jobs/s",
        "n_gpus": 1,
        "steps": len(table),
        "warmup": 1,
        "ms_per_step": mean_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": SERVE_CLASSES_WORKLOAD, "edge_factor": 16,
                   "mix_scales_covered": [10, top],
                   "classes": {f"({r},{s}) s{sc}": v for (r, s, sc), v in sorted(table.items())},
                   "not_measured": [f"({r},{s}) s{sc}" for r, s in only
                                    for sc in range(10, 21) if (r, s, sc) not in table],
                   "failed": failed,
                   "cap_s": args.class_cap_s},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
