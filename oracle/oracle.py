"""CPU oracle for (r,s) nucleus decomposition -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``nd_oracle.c`` (plain sequential C, no code shared
with the GPU library).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this module.

Functions follow the paper: Section 2 (definition of the (r,s)-clique core
number), Algorithm 1 (clique listing, here in plain lexicographic recursion),
Algorithm 2 (Count-Func, Update, Update-Func and the bucket loop).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nd_oracle.c")
_LIB = os.path.join(_HERE, "libnd_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.ndo_decompose.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(P)]
        lib.ndo_decompose.restype = ctypes.c_int
        lib.ndo_count.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(P)]
        lib.ndo_count.restype = ctypes.c_int
        lib.ndo_validate.argtypes = [ctypes.c_int32, P, P]
        lib.ndo_validate.restype = ctypes.c_int
        lib.ndo_count_one.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, ctypes.c_int, P]
        lib.ndo_count_one.restype = ctypes.c_uint64
        lib.ndo_support_at.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, ctypes.c_int, P, P, P,
                                       P, ctypes.c_uint64]
        lib.ndo_support_at.restype = ctypes.c_int64
        for name in ("ndo_n_s", "ndo_rounds", "ndo_discoveries", "ndo_decrements",
                     "ndo_max_kappa"):
            getattr(lib, name).argtypes = [P]
            getattr(lib, name).restype = ctypes.c_uint64
        lib.ndo_n_r.argtypes = [P]
        lib.ndo_n_r.restype = ctypes.c_int64
        lib.ndo_copy.argtypes = [P, P, P, P]
        lib.ndo_copy.restype = None
        lib.ndo_copy_final.argtypes = [P, P]
        lib.ndo_copy_final.restype = None
        lib.ndo_copy_rounds.argtypes = [P, P, P]
        lib.ndo_copy_rounds.restype = None
        lib.ndo_free.argtypes = [P]
        lib.ndo_free.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        names = {1: "EINVAL", 2: "EGRAPH", 5: "ENOMEM"}
        super().__init__(f"oracle error {code} ({names.get(code, '?')})")
        self.code = code


@dataclass
class OracleResult:
    r: int
    s: int
    rcliques: np.ndarray      # int32[n_r, r], rows ascending, lexicographic order
    counts: np.ndarray        # uint64[n_r] initial s-clique counts
    kappa: np.ndarray | None  # uint64[n_r] nucleus numbers
    final_counts: np.ndarray | None  # uint64[n_r] counts after peeling
    n_s: int
    rounds: int
    round_sizes: np.ndarray   # uint64[rounds]
    round_k: np.ndarray       # uint64[rounds]
    discoveries: int
    decrements: int
    max_kappa: int

    @property
    def n_r(self) -> int:
        return int(self.rcliques.shape[0])


def _graph_arrays(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return rp, cl


def _collect(lib, h, r, s, with_peel: bool) -> OracleResult:
    n_r = lib.ndo_n_r(h)
    tup = np.zeros(max(n_r * r, 1), dtype=np.int32)
    cnt = np.zeros(max(n_r, 1), dtype=np.uint64)
    kap = np.zeros(max(n_r, 1), dtype=np.uint64) if with_peel else None
    fin = np.zeros(max(n_r, 1), dtype=np.uint64) if with_peel else None
    lib.ndo_copy(h, _ptr(tup), _ptr(cnt), _ptr(kap) if kap is not None else None)
    if fin is not None:
        lib.ndo_copy_final(h, _ptr(fin))
    rounds = lib.ndo_rounds(h) if with_peel else 0
    rs = np.zeros(max(rounds, 1), dtype=np.uint64)
    rk = np.zeros(max(rounds, 1), dtype=np.uint64)
    if rounds:
        lib.ndo_copy_rounds(h, _ptr(rs), _ptr(rk))
    return OracleResult(
        r=r, s=s,
        rcliques=tup[: n_r * r].reshape(n_r, r),
        counts=cnt[:n_r],
        kappa=kap[:n_r] if kap is not None else None,
        final_counts=fin[:n_r] if fin is not None else None,
        n_s=int(lib.ndo_n_s(h)),
        rounds=int(rounds),
        round_sizes=rs[:rounds],
        round_k=rk[:rounds],
        discoveries=int(lib.ndo_discoveries(h)) if with_peel else 0,
        decrements=int(lib.ndo_decrements(h)) if with_peel else 0,
        max_kappa=int(lib.ndo_max_kappa(h)) if with_peel else 0,
    )


def decompose(n: int, row_ptr, col, r: int, s: int, single: bool = False) -> OracleResult:
    """Full (r,s) nucleus decomposition.  ``single`` selects one-at-a-time
    peeling (no rounds recorded) instead of bulk rounds."""
    lib = _load()
    rp, cl = _graph_arrays(row_ptr, col)
    h = ctypes.c_void_p()
    rc = lib.ndo_decompose(int(n), _ptr(rp), _ptr(cl), int(r), int(s), int(bool(single)),
                           ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    try:
        return _collect(lib, h, r, s, True)
    finally:
        lib.ndo_free(h)


def count(n: int, row_ptr, col, r: int, s: int) -> OracleResult:
    """r-clique table and initial s-clique counts only (Count-Func)."""
    lib = _load()
    rp, cl = _graph_arrays(row_ptr, col)
    h = ctypes.c_void_p()
    rc = lib.ndo_count(int(n), _ptr(rp), _ptr(cl), int(r), int(s), ctypes.byref(h))
    if rc:
        raise OracleError(rc)
    try:
        return _collect(lib, h, r, s, False)
    finally:
        lib.ndo_free(h)


def validate(n: int, row_ptr, col) -> int:
    lib = _load()
    rp, cl = _graph_arrays(row_ptr, col)
    return int(lib.ndo_validate(int(n), _ptr(rp), _ptr(cl)))


def count_one(n: int, row_ptr, col, r: int, s: int, R) -> int:
    """Number of s-cliques containing the r-clique R (sorted original ids)."""
    lib = _load()
    rp, cl = _graph_arrays(row_ptr, col)
    Rv = np.ascontiguousarray(sorted(int(x) for x in R), dtype=np.int32)
    return int(lib.ndo_count_one(int(n), _ptr(rp), _ptr(cl), int(r), int(s), _ptr(Rv)))


def _pack(cols, bits):
    key = np.zeros(cols[0].shape[0], dtype=np.uint64)
    for c in cols:
        key = (key << np.uint64(bits)) | c.astype(np.uint64)
    return key


def _kappa_lex_order(rc: np.ndarray, n: int) -> np.ndarray:
    """Row order of rc sorted lexicographically; vertex ids are packed into
    at most two 64-bit keys so large tables sort in one or two passes."""
    m, r = rc.shape
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    bits = max(1, int(n - 1).bit_length())
    per = 64 // bits
    if r <= per:
        return np.argsort(_pack([rc[:, i] for i in range(r)], bits), kind="stable")
    if r <= 2 * per:
        hi = _pack([rc[:, i] for i in range(per)], bits)
        lo = _pack([rc[:, i] for i in range(per, r)], bits)
        return np.lexsort((lo, hi))
    return np.lexsort(rc.T[::-1])


class KappaTable:
    """A kappa assignment over r-cliques, sorted for lookup by the local
    certificate (the assignment under test may come from anywhere)."""

    def __init__(self, n: int, rcliques: np.ndarray, kappa: np.ndarray):
        rc = np.sort(np.asarray(rcliques, dtype=np.int32), axis=1)
        order = _kappa_lex_order(rc, n)
        self.tab = np.ascontiguousarray(rc[order], dtype=np.int32)
        self.kap = np.ascontiguousarray(np.asarray(kappa)[order], dtype=np.uint32)
        first = np.zeros(n + 1, dtype=np.int64)
        if self.tab.shape[0]:
            np.cumsum(np.bincount(self.tab[:, 0], minlength=n), out=first[1:])
        self.first = first
        self.n = n


def support_at(n: int, row_ptr, col, r: int, s: int, table: KappaTable, R, threshold: int) -> int:
    """#{S containing R : every r-subset R' of S other than R has kappa(R') >=
    threshold}, using the kappa values of ``table``."""
    lib = _load()
    rp, cl = _graph_arrays(row_ptr, col)
    Rv = np.ascontiguousarray(sorted(int(x) for x in R), dtype=np.int32)
    tab = table.tab if table.tab.size else np.zeros((1, r), dtype=np.int32)
    kap = table.kap if table.kap.size else np.zeros(1, dtype=np.uint32)
    v = lib.ndo_support_at(int(n), _ptr(rp), _ptr(cl), int(r), int(s), _ptr(tab),
                           _ptr(table.first), _ptr(kap), _ptr(Rv), int(threshold))
    if v < 0:
        raise OracleError(1)
    return int(v)
