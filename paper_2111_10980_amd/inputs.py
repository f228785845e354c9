"""Seeded synthetic graph generators (input recipes only).

This module builds the graphs that both the GPU path and the CPU oracle
consume.  It holds none of the decomposition's arithmetic: it only draws
edges from a seeded ``numpy.random.default_rng`` (PCG64) and writes a
canonical CSR (int64 ``row_ptr[n+1]``, int32 ``col[2m]``; every row strictly
ascending, symmetric, no self-loops, no duplicates).

The graph families stand in for the paper's benchmark inputs (its SNAP graphs
are not used here) and follow the synthetic workloads the decomposition is
measured on: Erdos-Renyi G(n, m), rMAT (the paper's Section 5.1 uses rMAT with
its own a..d; the quadrant probabilities are arguments here), Chung-Lu
power-law graphs with planted cliques, batches of small uneven graphs and a
Poisson stream of serving jobs.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class CSR:
    """Canonical undirected simple graph in CSR form (host numpy arrays)."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[2m]

    @property
    def m(self) -> int:
        return int(self.col.shape[0]) // 2

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr_from_edges(n: int, u, v) -> CSR:
    """Symmetrise an edge list, drop self-loops and duplicates, sort rows."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    # both arc directions, ordered by (src, dst): the keys are distinct
    arcs = np.concatenate([key, hi * np.int64(n) + lo])
    arcs.sort()
    src = arcs // n
    dst = arcs % n
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n=n, row_ptr=row_ptr, col=dst.astype(np.int32))


def edges_of(g: CSR):
    """Undirected edge list (u < v) of a CSR graph."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    keep = src < dst
    return src[keep], dst[keep]


# --------------------------------------------------------------------------
# Families
# --------------------------------------------------------------------------

def erdos_renyi(n: int, m: int, seed: int) -> CSR:
    """G(n, m): uniform pairs u != v drawn until m distinct undirected edges."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = np.random.default_rng(seed)
    have = np.empty(0, dtype=np.int64)
    while have.size < m:
        need = m - have.size
        batch = max(2 * need, 1024)
        a = rng.integers(0, n, size=batch, dtype=np.int64)
        b = rng.integers(0, n, size=batch, dtype=np.int64)
        ok = a != b
        a, b = a[ok], b[ok]
        key = np.minimum(a, b) * n + np.maximum(a, b)
        allk = np.concatenate([have, key])
        _, first = np.unique(allk, return_index=True)
        first.sort()  # keep first-drawn order
        have = allk[first][:m]
    lo, hi = have // n, have % n
    return csr_from_edges(n, lo, hi)


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
         d=0.05, permute: bool = True) -> CSR:
    """rMAT: 2^scale vertices, edge_factor * 2^scale draws.

    Each draw picks one quadrant per bit with probabilities (a, b, c, d),
    then a seeded vertex permutation hides the hub ids; the result is
    symmetrised with self-loops and duplicates removed.
    """
    s = float(a + b + c + d)
    a, b, c = a / s, b / s, c / s
    n = 1 << scale
    ne = edge_factor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(ne, dtype=np.int64)
    dst = np.zeros(ne, dtype=np.int64)
    for bit in range(scale):
        x = rng.random(ne)
        sbit = x >= (a + b)  # quadrants c, d set the source bit
        dbit = ((x >= a) & (x < a + b)) | (x >= a + b + c)  # quadrants b, d
        src |= sbit.astype(np.int64) << bit
        dst |= dbit.astype(np.int64) << bit
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src, dst = perm[src], perm[dst]
    return csr_from_edges(n, src, dst)


def _chung_lu_weights(n: int, avg_deg: float, beta: float) -> np.ndarray:
    """w_i = w_max * (i0 / (i + i0))^(1/(beta-1)), i0 solved so mean(w) = avg_deg."""
    w_max = np.sqrt(n * avg_deg)
    gamma = 1.0 / (beta - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def mean_w(i0):
        return float(np.mean(w_max * (i0 / (idx + i0)) ** gamma))

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_w(mid) < avg_deg:
            lo = mid
        else:
            hi = mid
    i0 = 0.5 * (lo + hi)
    return w_max * (i0 / (idx + i0)) ** gamma


def chung_lu_planted(n: int, avg_deg: float, beta: float, n_cliques: int,
                     kmin: int, kmax: int, seed: int) -> CSR:
    """Chung-Lu power-law graph plus planted cliques on random vertex sets.

    n*avg_deg/2 endpoint pairs are drawn independently with probability
    proportional to the weights ("ball dropping"); loops and duplicates are
    dropped; ids are permuted; then ``n_cliques`` cliques of size uniform in
    [kmin, kmax] are added on uniformly random vertex sets.
    """
    rng = np.random.default_rng(seed)
    w = _chung_lu_weights(n, avg_deg, beta)
    p = w / w.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    ne = int(round(n * avg_deg / 2))
    u = np.searchsorted(cdf, rng.random(ne), side="right").astype(np.int64)
    v = np.searchsorted(cdf, rng.random(ne), side="right").astype(np.int64)
    perm = rng.permutation(n).astype(np.int64)
    u, v = perm[u], perm[v]
    us, vs = [u], [v]
    for _ in range(n_cliques):
        k = int(rng.integers(kmin, kmax + 1))
        k = min(k, n)
        verts = rng.choice(n, size=k, replace=False).astype(np.int64)
        iu, iv = np.triu_indices(k, 1)
        us.append(verts[iu])
        vs.append(verts[iv])
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def planted_er(n: int, avg_deg: float, n_cliques: int, kmin: int, kmax: int,
               seed: int) -> CSR:
    """ER base G(n, round(n*d/2)) plus planted cliques (batched workload)."""
    rng = np.random.default_rng(seed)
    m = min(int(round(n * avg_deg / 2)), n * (n - 1) // 2)
    base = erdos_renyi(n, m, int(rng.integers(0, 2**62)))
    bu, bv = edges_of(base)
    us, vs = [bu], [bv]
    for _ in range(n_cliques):
        k = min(int(rng.integers(kmin, kmax + 1)), n)
        verts = rng.choice(n, size=k, replace=False).astype(np.int64)
        iu, iv = np.triu_indices(k, 1)
        us.append(verts[iu])
        vs.append(verts[iv])
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def sparse_with_dense_block(n: int, avg_deg: float, block: int, p: float,
                            n_cliques: int, kmin: int, kmax: int, seed: int) -> CSR:
    """A sparse ER graph G(n, round(n*d/2)) with a dense part: ``block`` vertex
    ids drawn uniformly from [0, n) carry G(block, p) among themselves plus
    ``n_cliques`` overlapping cliques of size uniform in [kmin, kmax] on
    random subsets of the block.  Large n with the cliques concentrated on a
    few hundred vertices (which get the top ranks of a degree order)."""
    rng = np.random.default_rng(seed)
    base = erdos_renyi(n, int(round(n * avg_deg / 2)), int(rng.integers(0, 2**62)))
    bu, bv = edges_of(base)
    ids = rng.choice(n, size=block, replace=False).astype(np.int64)
    iu, iv = np.triu_indices(block, 1)
    keep = rng.random(iu.size) < p
    us, vs = [bu, ids[iu[keep]]], [bv, ids[iv[keep]]]
    for _ in range(n_cliques):
        k = min(int(rng.integers(kmin, kmax + 1)), block)
        verts = ids[rng.choice(block, size=k, replace=False)]
        cu, cv = np.triu_indices(k, 1)
        us.append(verts[cu])
        vs.append(verts[cv])
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def complete_graph(n: int) -> CSR:
    iu, iv = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, iv)


def disjoint_union(graphs) -> CSR:
    us, vs, off = [], [], 0
    for g in graphs:
        a, b = edges_of(g)
        us.append(a + off)
        vs.append(b + off)
        off += g.n
    if not us:
        return csr_from_edges(0, [], [])
    return csr_from_edges(off, np.concatenate(us), np.concatenate(vs))


def permute(g: CSR, seed: int) -> tuple[CSR, np.ndarray]:
    """Relabel vertices by a seeded permutation; returns (graph, perm) with
    new id = perm[old id]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.n).astype(np.int64)
    a, b = edges_of(g)
    return csr_from_edges(g.n, perm[a], perm[b]), perm


# The worked example of the paper's Section 3.2 (figure "nd-example"):
# vertices a..g = 0..6, a 5-clique on {a,b,c,d,e} plus af, bf, ef, cg, dg.
EXAMPLE_NAMES = "abcdefg"


def worked_example() -> CSR:
    k5 = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    extra = [(0, 5), (1, 5), (4, 5), (2, 6), (3, 6)]
    e = np.array(k5 + extra, dtype=np.int64)
    return csr_from_edges(7, e[:, 0], e[:, 1])


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def er_2000(seed: int = 1) -> CSR:
    """Erdos-Renyi G(n=2,000, m=10,000); the (2,3) workload."""
    return erdos_renyi(2000, 10000, seed)


def rmat_paper(scale: int, edge_factor: int, seed: int) -> CSR:
    """rMAT with the paper's own parameters (a, b, c, d) = (.5, .1, .1, .3)
    (Section 5.1), used for its density sweep over edge factors."""
    return rmat(scale, edge_factor, seed, a=0.5, b=0.1, c=0.1, d=0.3)


# the density sweep: scale 16, edge factor 4..32, seed 5000 + edge factor
DENSITY_SWEEP_SCALE = 16
DENSITY_SWEEP_EF = (4, 8, 16, 32)
DENSITY_SWEEP_RS = ((2, 3), (3, 4), (4, 5))


def rmat18(seed: int = 18) -> CSR:
    """rMAT scale 18, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05); the (3,4)
    single-graph workload."""
    return rmat(18, 16, seed)


def chung_lu_1m(seed: int = 2021) -> CSR:
    """Chung-Lu n=1,000,000, average degree 20, exponent 2.1, plus 200 planted
    cliques of size uniform in [20, 60]; the (4,5) and (2,4) workload."""
    return chung_lu_planted(1_000_000, 20.0, 2.1, 200, 20, 60, seed)


def batch_graph(i: int) -> CSR:
    """Graph i of the batched workload: n ~ U{50..5000}; i < 2048 plain ER
    with average degree ~U[8,30]; i >= 2048 the same base plus 1-5 planted
    cliques of size ~U{10..40}."""
    rng = np.random.default_rng(10_000 + i)
    n = int(rng.integers(50, 5001))
    d = float(rng.uniform(8.0, 30.0))
    if i < 2048:
        m = min(int(round(n * d / 2)), n * (n - 1) // 2)
        return erdos_renyi(n, m, int(rng.integers(0, 2**62)))
    q = int(rng.integers(1, 6))
    return planted_er(n, d, q, 10, 40, int(rng.integers(0, 2**62)))


def batch_order(count: int = 4096, seed: int = 4096) -> np.ndarray:
    """Shuffled processing order of the batched workload."""
    return np.random.default_rng(seed).permutation(count)


@dataclass(frozen=True)
class Job:
    arrival_s: float
    scale: int
    edge_factor: int
    r: int
    s: int
    graph_seed: int


def serving_stream(rate_per_s: float, n_jobs: int, seed: int = 7,
                   min_scale: int = 10, max_scale: int = 20) -> list[Job]:
    """Poisson arrivals of (rMAT graph, r, s) jobs: scale ~U{min..max},
    edge factor ~U{8..16}, r ~U{1,2,3}, s ~U{r+1, r+2}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for _ in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        scale = int(rng.integers(min_scale, max_scale + 1))
        ef = int(rng.integers(8, 17))
        r = int(rng.integers(1, 4))
        s = r + int(rng.integers(1, 3))
        jobs.append(Job(t, scale, ef, r, s, int(rng.integers(0, 2**31))))
    return jobs
