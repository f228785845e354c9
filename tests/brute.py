"""Brute-force references for tiny graphs (pure Python, test-only).

Each function restates a definition from the paper directly, with no shared
code with either the oracle or the GPU library:

* ``kappa_by_subsets``  -- the (r,s)-clique core number of Section 2 taken
  literally: the largest c such that some set X of r-cliques containing R has
  every member in at least c s-cliques whose r-subsets all lie in X.  Every
  subset X of the r-cliques is tried, so it is only for |K_r| <= ~14.
* ``kappa_by_cores``    -- the same quantity through the c-cores: for each c,
  repeatedly discard r-cliques with fewer than c surviving s-cliques; what is
  left is the largest feasible set at level c.
* ``kappa_by_hindex``   -- the local model the paper compares against in
  Section 1 and Section 5: iterate tau(R) <- H({min over the other r-subsets
  R' of S of tau(R') : S contains R}) from the initial counts until nothing
  changes; it converges to the same numbers.
* ``rounds_by_recount`` -- the bulk rounds of Algorithm 2 with every count
  recomputed from scratch each round (no decrements, no owner rule): a live
  r-clique's count is the number of its s-cliques with no peeled r-subset.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np


def adjacency(n, row_ptr, col):
    adj = [set() for _ in range(n)]
    for v in range(n):
        for i in range(int(row_ptr[v]), int(row_ptr[v + 1])):
            adj[v].add(int(col[i]))
    return adj


def cliques(n, adj, c):
    out = []

    def rec(cur, cand):
        if len(cur) == c:
            out.append(tuple(cur))
            return
        for i, x in enumerate(cand):
            rec(cur + [x], [y for y in cand[i + 1:] if y in adj[x]])

    rec([], list(range(n)))
    return out


def structure(n, row_ptr, col, r, s):
    adj = adjacency(n, row_ptr, col)
    Kr = cliques(n, adj, r)
    Ks = cliques(n, adj, s)
    idx = {R: i for i, R in enumerate(Kr)}
    subs = [[idx[t] for t in combinations(S, r)] for S in Ks]
    contains = [[] for _ in Kr]
    for j, sb in enumerate(subs):
        for i in sb:
            contains[i].append(j)
    return Kr, Ks, subs, contains


def counts(n, row_ptr, col, r, s):
    Kr, Ks, subs, contains = structure(n, row_ptr, col, r, s)
    return Kr, [len(c) for c in contains]


def kappa_by_subsets(n, row_ptr, col, r, s):
    Kr, Ks, subs, contains = structure(n, row_ptr, col, r, s)
    nr = len(Kr)
    if nr > 16:
        raise ValueError("too many r-cliques for subset enumeration")
    kap = [0] * nr
    for mask in range(1, 1 << nr):
        members = [i for i in range(nr) if mask >> i & 1]
        inside = [all(mask >> i & 1 for i in sb) for sb in subs]
        d = [sum(1 for j in contains[i] if inside[j]) for i in members]
        c = min(d)
        for i in members:
            if c > kap[i]:
                kap[i] = c
    return Kr, kap


def kappa_by_cores(n, row_ptr, col, r, s):
    Kr, Ks, subs, contains = structure(n, row_ptr, col, r, s)
    nr = len(Kr)
    kap = [0] * nr
    c = 1
    while True:
        alive = [True] * nr
        changed = True
        while changed:
            changed = False
            for i in range(nr):
                if not alive[i]:
                    continue
                d = sum(1 for j in contains[i] if all(alive[x] for x in subs[j]))
                if d < c:
                    alive[i] = False
                    changed = True
        if not any(alive):
            break
        for i in range(nr):
            if alive[i]:
                kap[i] = c
        c += 1
    return Kr, kap


def _h_index(values):
    vals = sorted(values, reverse=True)
    h = 0
    for i, v in enumerate(vals):
        if v >= i + 1:
            h = i + 1
        else:
            break
    return h


def kappa_by_hindex(n, row_ptr, col, r, s, max_iters=10_000):
    Kr, Ks, subs, contains = structure(n, row_ptr, col, r, s)
    tau = [len(c) for c in contains]
    for _ in range(max_iters):
        new = []
        for i in range(len(Kr)):
            vals = [min(tau[x] for x in subs[j] if x != i) for j in contains[i]]
            new.append(_h_index(vals))
        if new == tau:
            return Kr, tau
        tau = new
    raise RuntimeError("h-index iteration did not converge")


def rounds_by_recount(n, row_ptr, col, r, s):
    """Returns (Kr, kappa, round sizes, round levels)."""
    Kr, Ks, subs, contains = structure(n, row_ptr, col, r, s)
    nr = len(Kr)
    peeled = [False] * nr
    kap = [0] * nr
    sizes, levels = [], []
    k = 0
    while not all(peeled):
        live = [i for i in range(nr) if not peeled[i]]
        cnt = {i: sum(1 for j in contains[i] if not any(peeled[x] for x in subs[j])) for i in live}
        k = max(k, min(cnt.values()))
        A = [i for i in live if cnt[i] <= k]
        for i in A:
            peeled[i] = True
            kap[i] = k
        sizes.append(len(A))
        levels.append(k)
    return Kr, kap, sizes, levels


def as_dict(Kr, values):
    return {tuple(R): int(v) for R, v in zip(Kr, values)}


def rows_dict(rcliques, values):
    return {tuple(int(x) for x in sorted(row)): int(v) for row, v in zip(np.asarray(rcliques), values)}
