"""MI355X (gfx950) (r,s) nucleus decomposition -- Python binding.

A thin ctypes layer over the C ABI in ``include/nd.h``: the functions below
carry the ABI's names and only marshal arguments (torch tensors give device
pointers and the HIP stream).  Every step of the decomposition runs in the
library's HIP kernels; there is no CPU fallback: the first call raises
ImportError if the built library ``libnd.so`` is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnd.so")

ND_MAX_S = 8
ND_ENOMEM = 5
WS_ALIGN = 256
STATUS = {0: "ND_OK", 1: "ND_EINVAL", 2: "ND_EGRAPH", 3: "ND_EKEYWIDTH", 4: "ND_EOVERFLOW",
          5: "ND_ENOMEM", 6: "ND_EHIP", 7: "ND_ESTATE"}
PHASES = ("validate", "orient", "table", "count", "bucket", "peel", "emit", "total")


class NdError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class nd_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p)]


class nd_options(ctypes.Structure):
    _fields_ = [("orient", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("load_factor", ctypes.c_float), ("path", ctypes.c_int32),
                ("canonical", ctypes.c_int32), ("trace_cap", ctypes.c_uint32),
                ("record_cap", ctypes.c_uint64), ("debug_count_bias", ctypes.c_uint64),
                ("queue_depth", ctypes.c_int32), ("contract", ctypes.c_int32),
                ("graph_rounds", ctypes.c_int32), ("levels", ctypes.c_int32)]


ND_TUNE_MAX = 16


class nd_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("best", ctypes.c_int32),
                ("sample_graphs", ctypes.c_int32), ("opt", nd_options * ND_TUNE_MAX),
                ("ms", ctypes.c_float * ND_TUNE_MAX)]


class nd_roofline(ctypes.Structure):
    _fields_ = [("copy_gbs", ctypes.c_double), ("gather16_gops", ctypes.c_double),
                ("atomic_ret_gops", ctypes.c_double), ("atomic_noret_gops", ctypes.c_double)]


class nd_stats(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_uint64), ("n_s", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("k_advances", ctypes.c_uint64), ("decrements", ctypes.c_uint64),
                ("discoveries", ctypes.c_uint64), ("table_slots", ctypes.c_uint64),
                ("max_kappa", ctypes.c_uint32), ("max_out_degree", ctypes.c_uint32),
                ("ms", ctypes.c_float * 8), ("count_kernel_ms", ctypes.c_float),
                ("peel_kernel_ms", ctypes.c_float), ("count_launches", ctypes.c_uint32),
                ("peel_launches", ctypes.c_uint32), ("atomics", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("max_round_records", ctypes.c_uint64),
                ("max_round_arcs", ctypes.c_uint64), ("contractions", ctypes.c_uint32),
                ("key_words", ctypes.c_uint32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run paper_2111_10980_amd.build.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.nd_plan_create.argtypes = [ctypes.POINTER(nd_csr), ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(nd_options), ctypes.c_uint64, P,
                                   ctypes.POINTER(P)]
    lib.nd_plan_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
    lib.nd_run.argtypes = [P, P, ctypes.c_uint64, P, P, P, ctypes.POINTER(nd_stats)]
    lib.nd_run_noalloc.argtypes = [P, P, P, P, ctypes.POINTER(nd_stats)]
    lib.nd_round_trace.argtypes = [P, P, P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.nd_plan_destroy.argtypes = [P]
    lib.nd_release_cached.argtypes = []
    lib.nd_roofline_measure.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P,
                                        ctypes.POINTER(nd_roofline)]
    lib.nd_roofline_measure.restype = ctypes.c_int
    lib.nd_batch_create.argtypes = [ctypes.POINTER(nd_csr), ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(nd_options), ctypes.c_uint64, P,
                                    ctypes.POINTER(P)]
    lib.nd_batch_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]
    lib.nd_batch_run.argtypes = [P, P, ctypes.c_uint64, P, P, P, P, ctypes.POINTER(nd_stats)]
    lib.nd_batch_round_trace.argtypes = [P, P, P, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_uint64)]
    lib.nd_batch_destroy.argtypes = [P]
    lib.nd_batch_autotune.argtypes = [ctypes.POINTER(nd_csr), ctypes.c_int32, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(nd_options), ctypes.c_int32,
                                      P, ctypes.POINTER(nd_options),
                                      ctypes.POINTER(nd_tune_report)]
    for name in ("nd_batch_create", "nd_batch_sizes", "nd_batch_run", "nd_batch_round_trace",
                 "nd_batch_destroy", "nd_batch_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    lib.nd_server_create.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(P)]
    lib.nd_server_submit.argtypes = [P, ctypes.POINTER(nd_csr), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(nd_options), P,
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.nd_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.nd_server_result.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(nd_stats), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.nd_server_copy.argtypes = [P, ctypes.c_uint64, P, P]
    lib.nd_server_release.argtypes = [P, ctypes.c_uint64]
    lib.nd_server_destroy.argtypes = [P]
    for name in ("nd_server_create", "nd_server_submit", "nd_server_wait", "nd_server_result",
                 "nd_server_copy", "nd_server_release", "nd_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    lib.nd_status_str.argtypes = [ctypes.c_int]
    lib.nd_status_str.restype = ctypes.c_char_p
    lib.nd_last_error.argtypes = []
    lib.nd_last_error.restype = ctypes.c_char_p
    for name in ("nd_plan_create", "nd_plan_sizes", "nd_run", "nd_run_noalloc",
                 "nd_round_trace", "nd_plan_destroy", "nd_release_cached"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


class _Lazy:
    """Loads libnd.so on first use; raises ImportError if it is not built."""

    _h = None

    def __getattr__(self, name):
        if _Lazy._h is None:
            _Lazy._h = _load()
        return getattr(_Lazy._h, name)


_lib = _Lazy()


def library():
    """The loaded ctypes library (raises ImportError when it is not built)."""
    if _Lazy._h is None:
        _Lazy._h = _load()
    return _Lazy._h

EXPORTED = ("nd_plan_create", "nd_plan_sizes", "nd_run", "nd_run_noalloc", "nd_round_trace",
            "nd_plan_destroy",
            "nd_release_cached", "nd_status_str", "nd_last_error", "nd_roofline_measure",
            "nd_batch_create", "nd_batch_sizes", "nd_batch_run", "nd_batch_round_trace",
            "nd_batch_destroy", "nd_batch_autotune", "nd_server_create", "nd_server_submit", "nd_server_wait",
            "nd_server_result", "nd_server_copy", "nd_server_release", "nd_server_destroy")


def _check(rc: int):
    if rc != 0:
        raise NdError(rc, _lib.nd_last_error().decode(errors="replace"))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ raw ABI

def make_options(orient: int = 0, timing: bool = False, load_factor: float = 0.0,
                 generic: bool = False, canonical: bool = False, trace_cap: int = 0,
                 record_cap: int = 0, debug_count_bias: int = 0, queue_depth: int = 0,
                 graph_rounds: bool = False, contract: bool = False,
                 levels: int = 0) -> nd_options:
    return nd_options(int(orient), int(bool(timing)), float(load_factor), int(bool(generic)),
                      int(bool(canonical)), int(trace_cap), int(record_cap),
                      int(debug_count_bias), int(queue_depth), int(bool(contract)),
                      int(bool(graph_rounds)), int(levels))


def nd_plan_create(row_ptr, col, r: int, s: int, orient: int = 0, load_factor: float = 0.0,
                   hbm_budget_bytes: int = 0, stream=None, timing: bool = False,
                   generic: bool = False, canonical: bool = False, trace_cap: int = 0,
                   record_cap: int = 0, debug_count_bias: int = 0, queue_depth: int = 0,
                   graph_rounds: bool = False, contract: bool = False, levels: int = 0):
    """row_ptr (int64, n+1) and col (int32) are CUDA tensors; returns a plan handle."""
    import torch
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col int32")
    if not (row_ptr.is_cuda and (col.is_cuda or col.numel() == 0)):
        raise TypeError("row_ptr and col must be device tensors")
    row_ptr = row_ptr.contiguous()
    col = col.contiguous()
    g = nd_csr(int(row_ptr.numel() - 1), int(col.numel()), row_ptr.data_ptr(),
               col.data_ptr() if col.numel() else None)
    opt = make_options(orient, timing, load_factor, generic, canonical, trace_cap, record_cap,
                       debug_count_bias, queue_depth, graph_rounds, contract, levels)
    h = ctypes.c_void_p()
    _check(_lib.nd_plan_create(ctypes.byref(g), int(r), int(s), ctypes.byref(opt),
                               int(hbm_budget_bytes), _stream_handle(stream), ctypes.byref(h)))
    return h


def nd_plan_sizes(plan):
    """(n_r, workspace bytes a run needs, device bytes the plan holds)."""
    n_r = ctypes.c_uint64()
    ws = ctypes.c_uint64()
    held = ctypes.c_uint64()
    _check(_lib.nd_plan_sizes(plan, ctypes.byref(n_r), ctypes.byref(ws), ctypes.byref(held)))
    return int(n_r.value), int(ws.value), int(held.value)


def workspace(nbytes: int, device="cuda"):
    """A caller-owned device workspace (torch uint8, 256-byte aligned)."""
    import torch
    t = torch.empty(max(int(nbytes), 1) + WS_ALIGN, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % WS_ALIGN
    return t[off: off + max(int(nbytes), 1)]


def _ptr(t):
    return t.data_ptr() if t is not None and t.numel() else None


def nd_run(plan, ws, rcliques, kappa, counts=None, ws_bytes=None) -> dict:
    """ws: device workspace tensor (see workspace()); ws_bytes defaults to its size."""
    st = nd_stats()
    nbytes = int(ws.numel() * ws.element_size()) if ws_bytes is None else int(ws_bytes)
    _check(_lib.nd_run(plan, _ptr(ws), nbytes, _ptr(rcliques), _ptr(kappa), _ptr(counts),
                       ctypes.byref(st)))
    return stats_dict(st)


ND_NOALLOC_WORKSPACE_BYTES = 64 << 20


def nd_run_noalloc(plan, rcliques, kappa, counts=None) -> dict:
    """nd_run with the library's static device workspace (no allocation)."""
    st = nd_stats()
    _check(_lib.nd_run_noalloc(plan, _ptr(rcliques), _ptr(kappa), _ptr(counts),
                               ctypes.byref(st)))
    return stats_dict(st)


def nd_round_trace(plan):
    import numpy as np
    rounds = ctypes.c_uint64()
    _check(_lib.nd_round_trace(plan, None, None, 0, ctypes.byref(rounds)))
    n = int(rounds.value)
    sizes = np.zeros(max(n, 1), dtype=np.uint64)
    levels = np.zeros(max(n, 1), dtype=np.uint32)
    _check(_lib.nd_round_trace(plan, sizes.ctypes.data_as(ctypes.c_void_p),
                               levels.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(rounds)))
    return sizes[:n], levels[:n]


def nd_plan_destroy(plan):
    _check(_lib.nd_plan_destroy(plan))


def nd_batch_create(graphs, r: int, s: int, orient: int = 0, load_factor: float = 0.0,
                    hbm_budget_bytes: int = 0, stream=None, timing: bool = False,
                    generic: bool = False, canonical: bool = False, queue_depth: int = 0,
                    graph_rounds: bool = False):
    """graphs: sequence of (row_ptr int64, col int32) device tensor pairs."""
    arr = (nd_csr * max(1, len(graphs)))()
    keep = []
    for i, (rp, col) in enumerate(graphs):
        rp = rp.contiguous()
        col = col.contiguous()
        keep.append((rp, col))
        arr[i] = nd_csr(int(rp.numel() - 1), int(col.numel()), rp.data_ptr(),
                        col.data_ptr() if col.numel() else None)
    opt = make_options(orient, timing, load_factor, generic, canonical,
                       queue_depth=queue_depth, graph_rounds=graph_rounds)
    h = ctypes.c_void_p()
    _check(_lib.nd_batch_create(arr, len(graphs), int(r), int(s), ctypes.byref(opt),
                                int(hbm_budget_bytes), _stream_handle(stream), ctypes.byref(h)))
    return h


def nd_batch_sizes(batch):
    """(total rows, graph count, workspace bytes a batch run needs)."""
    n_r = ctypes.c_uint64()
    count = ctypes.c_int32()
    ws = ctypes.c_uint64()
    _check(_lib.nd_batch_sizes(batch, ctypes.byref(n_r), ctypes.byref(count), ctypes.byref(ws)))
    return int(n_r.value), int(count.value), int(ws.value)


def nd_batch_run(batch, ws, rcliques, kappa, counts=None):
    """Returns (row_offsets numpy uint64[count+1], stats dict)."""
    import numpy as np
    _, count, _ = nd_batch_sizes(batch)
    off = np.zeros(count + 1, dtype=np.uint64)
    st = nd_stats()
    _check(_lib.nd_batch_run(batch, _ptr(ws), int(ws.numel()), _ptr(rcliques), _ptr(kappa),
                             _ptr(counts), off.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(st)))
    return off, stats_dict(st)


def nd_batch_round_trace(batch):
    import numpy as np
    rounds = ctypes.c_uint64()
    _check(_lib.nd_batch_round_trace(batch, None, None, 0, ctypes.byref(rounds)))
    n = int(rounds.value)
    sizes = np.zeros(max(n, 1), dtype=np.uint64)
    levels = np.zeros(max(n, 1), dtype=np.uint32)
    _check(_lib.nd_batch_round_trace(batch, sizes.ctypes.data_as(ctypes.c_void_p),
                                     levels.ctypes.data_as(ctypes.c_void_p), n,
                                     ctypes.byref(rounds)))
    return sizes[:n], levels[:n]


def nd_batch_destroy(batch):
    _check(_lib.nd_batch_destroy(batch))


def _options_dict(o: nd_options) -> dict:
    return {name: getattr(o, name) for name, _ in nd_options._fields_}


def nd_batch_autotune(graphs, r: int, s: int, sample_count: int = 256, stream=None, **base):
    """Tunes orientation, queue depth and graph replay on a held-out sample of
    the graphs; returns (best options dict, report dict)."""
    arr = (nd_csr * max(1, len(graphs)))()
    keep = []
    for i, (rp, col) in enumerate(graphs):
        rp = rp.contiguous()
        col = col.contiguous()
        keep.append((rp, col))
        arr[i] = nd_csr(int(rp.numel() - 1), int(col.numel()), rp.data_ptr(),
                        col.data_ptr() if col.numel() else None)
    b = make_options(**base)
    best = nd_options()
    rep = nd_tune_report()
    _check(_lib.nd_batch_autotune(arr, len(graphs), int(r), int(s), ctypes.byref(b),
                                  int(sample_count), _stream_handle(stream), ctypes.byref(best),
                                  ctypes.byref(rep)))
    cands = [dict(_options_dict(rep.opt[i]), ms=float(rep.ms[i]))
             for i in range(rep.candidates)]
    return _options_dict(best), {"sample_graphs": int(rep.sample_graphs), "best": int(rep.best),
                                 "candidates": cands}


def nd_server_create(workers: int, hbm_budget_bytes: int = 0):
    h = ctypes.c_void_p()
    _check(_lib.nd_server_create(int(workers), int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def nd_server_submit(server, row_ptr, col, r: int, s: int, orient: int = 0,
                     generic: bool = False, stream=None) -> int:
    """The caller keeps row_ptr / col alive until the job is done.  The job
    waits for the work already queued on `stream` (default: torch's current
    stream), which produced the graph."""
    g = nd_csr(int(row_ptr.numel() - 1), int(col.numel()), row_ptr.data_ptr(),
               col.data_ptr() if col.numel() else None)
    opt = make_options(orient, generic=generic)
    job = ctypes.c_uint64()
    _check(_lib.nd_server_submit(server, ctypes.byref(g), int(r), int(s), ctypes.byref(opt),
                                 _stream_handle(stream), ctypes.byref(job)))
    return int(job.value)


def nd_server_wait(server, job: int, timeout_ms: int = -1) -> bool:
    done = ctypes.c_int32()
    _check(_lib.nd_server_wait(server, ctypes.c_uint64(job), int(timeout_ms), ctypes.byref(done)))
    return bool(done.value)


def nd_server_result(server, job: int, r: int, copy: bool = True):
    """(rcliques, kappa, stats, queue_ms, service_ms); with copy=True the
    device outputs are copied into new torch tensors."""
    import torch
    n_r = ctypes.c_uint64()
    rp = ctypes.c_void_p()
    kp = ctypes.c_void_p()
    st = nd_stats()
    qms = ctypes.c_double()
    sms = ctypes.c_double()
    _check(_lib.nd_server_result(server, ctypes.c_uint64(job), ctypes.byref(n_r),
                                 ctypes.byref(rp), ctypes.byref(kp), ctypes.byref(st),
                                 ctypes.byref(qms), ctypes.byref(sms)))
    n = int(n_r.value)
    rcl = kap = None
    if copy:
        rcl = torch.empty((n, r), dtype=torch.int32, device="cuda")
        kap = torch.empty((n,), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        nd_server_copy(server, job, rcl, kap)
    return rcl, kap, stats_dict(st), float(qms.value), float(sms.value)


def nd_server_copy(server, job: int, rcliques_dst, kappa_dst):
    """Device-to-device copy of a finished job's outputs into torch tensors."""
    _check(_lib.nd_server_copy(server, ctypes.c_uint64(job), ctypes.c_void_p(rcliques_dst.data_ptr()),
                               ctypes.c_void_p(kappa_dst.data_ptr())))


def nd_server_release(server, job: int):
    _check(_lib.nd_server_release(server, ctypes.c_uint64(job)))


def nd_server_destroy(server):
    _check(_lib.nd_server_destroy(server))


def nd_release_cached():
    _check(_lib.nd_release_cached())


def nd_status_str(code: int) -> str:
    return _lib.nd_status_str(int(code)).decode()


def nd_last_error() -> str:
    return _lib.nd_last_error().decode(errors="replace")


def nd_roofline_measure(table_bytes: int, count_bytes: int, stream=None) -> dict:
    """Measured device ceilings (include/nd_roofline.h)."""
    out = nd_roofline()
    rc = _lib.nd_roofline_measure(int(table_bytes), int(count_bytes), _stream_handle(stream),
                                  ctypes.byref(out))
    if rc != 0:
        raise NdError(rc, "roofline probe failed")
    return {name: float(getattr(out, name)) for name, _ in nd_roofline._fields_}


def stats_dict(st: nd_stats) -> dict:
    d = {name: getattr(st, name) for name, _ in nd_stats._fields_ if name != "ms"}
    d = {k: (float(v) if isinstance(v, float) else int(v)) for k, v in d.items()}
    d["ms"] = {ph: float(st.ms[i]) for i, ph in enumerate(PHASES)}
    return d


# --------------------------------------------------------------- convenience

@dataclass
class Decomposition:
    r: int
    s: int
    rcliques: object          # torch.int32 [n_r, r] (device), original ids ascending per row
    kappa: object             # torch.int32 view of uint32 [n_r] (device)
    counts: object | None     # initial s-clique counts [n_r] (device) or None
    stats: dict = field(default_factory=dict)
    round_sizes: object = None
    round_levels: object = None


def run_requery(plan, rcl, kap, cnt=None, device="cuda", attempts: int = 10):
    """nd_run with a workspace of the size nd_plan_sizes reports; when a
    round outgrows it (ND_ENOMEM and a larger reported size) the workspace is
    re-allocated and the plan run again.  Returns (stats, workspace bytes)."""
    for i in range(attempts):
        _, ws_bytes, _ = nd_plan_sizes(plan)
        ws = workspace(ws_bytes, device)
        try:
            return nd_run(plan, ws, rcl, kap, cnt, ws_bytes=ws_bytes), ws_bytes
        except NdError as e:
            _, again, _ = nd_plan_sizes(plan)
            if e.code != ND_ENOMEM or again <= ws_bytes or i + 1 == attempts:
                raise
        finally:
            del ws
    raise AssertionError("unreachable")


def decompose(row_ptr, col, r: int, s: int, with_counts: bool = False, orient: int = 0,
              load_factor: float = 0.0, hbm_budget_bytes: int = 0, stream=None,
              timing: bool = False, generic: bool = False, canonical: bool = False,
              trace_cap: int = 0, record_cap: int = 0, debug_count_bias: int = 0,
              queue_depth: int = 0, graph_rounds: bool = False, contract: bool = False,
              requery: bool = True, levels: int = 0) -> Decomposition:
    """Whole hot path on the current device: plan, workspace, run, round
    trace, destroy.  With requery a run whose round outgrew the workspace is
    repeated with the larger workspace the plan then reports."""
    import torch
    plan = nd_plan_create(row_ptr, col, r, s, orient, load_factor, hbm_budget_bytes, stream,
                          timing, generic, canonical, trace_cap, record_cap, debug_count_bias,
                          queue_depth, graph_rounds, contract, levels)
    try:
        n_r, ws_bytes, _ = nd_plan_sizes(plan)
        dev = row_ptr.device
        rcl = torch.empty((n_r, r), dtype=torch.int32, device=dev)
        kap = torch.empty((n_r,), dtype=torch.int32, device=dev)
        cnt = torch.empty((n_r,), dtype=torch.int32, device=dev) if with_counts else None
        if requery:
            stats, _ = run_requery(plan, rcl, kap, cnt, dev)
        else:
            ws = workspace(ws_bytes, dev)
            stats = nd_run(plan, ws, rcl, kap, cnt, ws_bytes=ws_bytes)
            del ws
        sizes, levels = nd_round_trace(plan)
    finally:
        nd_plan_destroy(plan)
    return Decomposition(r, s, rcl, kap, cnt, stats, sizes, levels)


@dataclass
class BatchDecomposition:
    r: int
    s: int
    rcliques: object          # int32 [n_r_total, r] device, graph-local ids
    kappa: object             # int32 view of uint32 [n_r_total] device
    counts: object | None
    row_offsets: object       # numpy uint64 [count+1]
    stats: dict = field(default_factory=dict)

    def graph(self, g: int):
        a, b = int(self.row_offsets[g]), int(self.row_offsets[g + 1])
        cnt = self.counts[a:b] if self.counts is not None else None
        return self.rcliques[a:b], self.kappa[a:b], cnt


def decompose_batch(graphs, r: int, s: int, with_counts: bool = False, orient: int = 0,
                    load_factor: float = 0.0, hbm_budget_bytes: int = 0, stream=None,
                    timing: bool = False, generic: bool = False,
                    canonical: bool = False, queue_depth: int = 0,
                    graph_rounds: bool = False) -> BatchDecomposition:
    """All graphs in one fused decomposition (graphs: (row_ptr, col) device pairs)."""
    import torch
    b = nd_batch_create(graphs, r, s, orient, load_factor, hbm_budget_bytes, stream, timing,
                        generic, canonical, queue_depth, graph_rounds)
    try:
        dev = graphs[0][0].device if graphs else torch.device("cuda")
        for i in range(10):
            n_r, _, ws_bytes = nd_batch_sizes(b)
            rcl = torch.empty((n_r, r), dtype=torch.int32, device=dev)
            kap = torch.empty((n_r,), dtype=torch.int32, device=dev)
            cnt = torch.empty((n_r,), dtype=torch.int32, device=dev) if with_counts else None
            ws = workspace(ws_bytes, dev)
            try:
                off, stats = nd_batch_run(b, ws, rcl, kap, cnt)
                break
            except NdError as e:  # a round outgrew the workspace: run again with more
                if e.code != ND_ENOMEM or nd_batch_sizes(b)[2] <= ws_bytes or i == 9:
                    raise
            finally:
                del ws
    finally:
        nd_batch_destroy(b)
    return BatchDecomposition(r, s, rcl, kap, cnt, off, stats)


@dataclass
class Served:
    job: int
    decomposition: Decomposition
    queue_ms: float      # submit -> start of service
    service_ms: float    # start -> end of service


class Server:
    """Continuous-batching request loop: jobs are admitted by the memory
    budget onto a pool of worker streams and run concurrently on the device.
    The graph tensors of a job are kept referenced until its result is taken."""

    def __init__(self, workers: int = 4, hbm_budget_bytes: int = 0):
        self.handle = nd_server_create(workers, hbm_budget_bytes)
        self._keep = {}

    def submit(self, row_ptr, col, r: int, s: int, orient: int = 0, generic: bool = False,
               stream=None) -> int:
        job = nd_server_submit(self.handle, row_ptr, col, r, s, orient, generic, stream)
        self._keep[job] = (row_ptr, col, r, s)
        return job

    def wait(self, job: int, timeout_ms: int = -1) -> bool:
        return nd_server_wait(self.handle, job, timeout_ms)

    def result(self, job: int) -> Served:
        """Wait for the job, copy its outputs into new tensors, free its
        device outputs; raises NdError with the job's own status if it failed."""
        _, _, r, s = self._keep[job]
        nd_server_wait(self.handle, job, -1)
        try:
            rcl, kap, stats, qms, sms = nd_server_result(self.handle, job, r, copy=True)
        finally:
            nd_server_release(self.handle, job)
            del self._keep[job]
        return Served(job, Decomposition(r, s, rcl, kap, None, stats), qms, sms)

    def close(self):
        if self.handle is not None:
            nd_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def to_device(g, device="cuda"):
    """Host CSR (inputs.CSR) -> (row_ptr, col) device tensors."""
    import torch
    rp = torch.from_numpy(g.row_ptr).to(device=device, dtype=torch.int64)
    col = torch.from_numpy(g.col).to(device=device, dtype=torch.int32)
    return rp, col
