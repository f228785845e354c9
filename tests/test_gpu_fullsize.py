"""GPU results at the full sizes of the measured workloads, in the launch
configuration bench.py times (default options, one decomposition of the
whole graph), checked on sampled r-cliques the oracle can verify one by one:

- the initial count of a sampled R equals the oracle's count of the
  s-cliques containing R (Algorithm 2, Count-Func);
- the nucleus number k of a sampled R satisfies the local certificate of a
  peeling result: at least k s-cliques containing R have every other
  r-subset at level >= k, and at most k have every other r-subset at level
  >= k+1 (Definition of the (r,s) nucleus; the fixed point the peel reaches);
- global identities: sum of counts = C(s,r) * n_s, and the table holds each
  r-clique once.

Samples mix uniform draws with the r-cliques of the highest levels, where the
deep rounds of the peel decide the value."""
from math import comb

import numpy as np
import pytest

from oracle import oracle
from paper_2111_10980_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _nd():
    import paper_2111_10980_amd as nd
    return nd


def check_sampled(g, r, s, n_uniform=40, n_top=24, seed=0):
    nd = _nd()
    rp, col = nd.to_device(g)
    print(f"[fullsize] n={g.n} m={g.m} r={r} s={s}", flush=True)
    d = nd.decompose(rp, col, r, s, with_counts=True)
    rcl = d.rcliques.cpu().numpy()
    kap = d.kappa.cpu().numpy().view(np.uint32)
    cnt = d.counts.cpu().numpy().view(np.uint32)
    n_r = rcl.shape[0]
    assert n_r == d.stats["n_r"]
    assert int(cnt.astype(np.uint64).sum()) == comb(s, r) * d.stats["n_s"]
    assert (np.diff(np.sort(rcl, axis=1), axis=1) > 0).all()  # r distinct vertices
    print(f"[fullsize] n_r={n_r} n_s={d.stats['n_s']} max kappa={int(kap.max())}; "
          "building the lookup table", flush=True)
    table = oracle.KappaTable(g.n, rcl, kap)
    assert (np.diff(table.tab, axis=0) != 0).any(axis=1).all()  # no r-clique twice
    rng = np.random.default_rng(seed)
    pick = list(rng.choice(n_r, size=min(n_uniform, n_r), replace=False))
    pick += list(np.argsort(kap, kind="stable")[-n_top:])
    for i in pick:
        R = [int(v) for v in rcl[i]]
        k = int(kap[i])
        assert oracle.count_one(g.n, g.row_ptr, g.col, r, s, R) == int(cnt[i]), R
        assert oracle.support_at(g.n, g.row_ptr, g.col, r, s, table, R, k) >= k, (R, k)
        assert oracle.support_at(g.n, g.row_ptr, g.col, r, s, table, R, k + 1) <= k, (R, k)
    return d


def test_rmat18_34_full():
    """rMAT scale 18, edge factor 16, (3,4): the single-graph workload."""
    check_sampled(inputs.rmat18(), 3, 4)


def test_chung_lu_1m_45_full():
    """Chung-Lu n = 1e6 with 200 planted cliques of 20-60 vertices, (4,5)."""
    check_sampled(inputs.chung_lu_1m(), 4, 5)


def test_chung_lu_1m_24_full():
    """The same graph, (2,4): edges of the planted cliques reach the deepest
    levels of the peel."""
    check_sampled(inputs.chung_lu_1m(), 2, 4)
