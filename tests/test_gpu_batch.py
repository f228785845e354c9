"""GPU parity of the batched decomposition (one fused run over many graphs)
against the CPU oracle, graph by graph."""
import numpy as np
import pytest

from oracle import oracle
from paper_2111_10980_amd import inputs

pytestmark = pytest.mark.gpu


def _nd():
    import paper_2111_10980_amd as nd
    return nd


def _canon(rcl, *vals):
    rcl = np.asarray(rcl)
    if rcl.shape[0] == 0:
        return (rcl,) + tuple(np.asarray(v) for v in vals)
    order = np.lexsort(rcl.T[::-1])
    return (rcl[order],) + tuple(np.asarray(v)[order] for v in vals)


def mixed_graphs(seed=0, count=40):
    rng = np.random.default_rng(seed)
    gs = [inputs.csr_from_edges(0, [], []), inputs.csr_from_edges(1, [], []),
          inputs.worked_example(), inputs.complete_graph(9), inputs.csr_from_edges(5, [], [])]
    while len(gs) < count:
        kind = int(rng.integers(0, 4))
        n = int(rng.integers(20, 300))
        sd = int(rng.integers(0, 2**31))
        if kind == 0:
            gs.append(inputs.erdos_renyi(n, min(n * (n - 1) // 2, int(n * rng.uniform(2, 8))), sd))
        elif kind == 1:
            gs.append(inputs.planted_er(n, float(rng.uniform(3, 9)), int(rng.integers(1, 4)), 5, 12,
                                        sd))
        elif kind == 2:
            gs.append(inputs.rmat(int(rng.integers(5, 9)), 8, sd))
        else:
            gs.append(inputs.complete_graph(int(rng.integers(2, 14))))
    order = rng.permutation(len(gs))
    return [gs[i] for i in order]


@pytest.mark.parametrize("r,s", [(3, 4), (2, 3), (1, 2), (2, 4), (4, 5)])
def test_batch_matches_oracle_per_graph(r, s):
    nd = _nd()
    gs = mixed_graphs(seed=r * 10 + s)
    dev = [nd.to_device(g) for g in gs]
    print(f"[batch] {len(gs)} graphs r={r} s={s}", flush=True)
    res = nd.decompose_batch(dev, r, s, with_counts=True)
    rcl = res.rcliques.cpu().numpy()
    kap = res.kappa.cpu().numpy().view(np.uint32)
    cnt = res.counts.cpu().numpy().view(np.uint32)
    off = res.row_offsets
    assert off[0] == 0 and off[-1] == rcl.shape[0]
    total_ns = 0
    for gi, g in enumerate(gs):
        a, b = int(off[gi]), int(off[gi + 1])
        ref = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
        grc, gk, gc = _canon(rcl[a:b], kap[a:b], cnt[a:b])
        assert grc.shape == ref.rcliques.shape, gi
        np.testing.assert_array_equal(grc, ref.rcliques)
        np.testing.assert_array_equal(gk.astype(np.uint64), ref.kappa)
        np.testing.assert_array_equal(gc.astype(np.uint64), ref.counts)
        total_ns += ref.n_s
    assert res.stats["n_s"] == total_ns


def test_batch_equals_single_runs():
    nd = _nd()
    gs = mixed_graphs(seed=7, count=12)
    dev = [nd.to_device(g) for g in gs]
    res = nd.decompose_batch(dev, 3, 4)
    rcl = res.rcliques.cpu().numpy()
    kap = res.kappa.cpu().numpy()
    for gi, (rp, col) in enumerate(dev):
        one = nd.decompose(rp, col, 3, 4)
        a, b = int(res.row_offsets[gi]), int(res.row_offsets[gi + 1])
        x = _canon(rcl[a:b], kap[a:b])
        y = _canon(one.rcliques.cpu().numpy(), one.kappa.cpu().numpy())
        for u, v in zip(x, y):
            np.testing.assert_array_equal(u, v)


def test_batch_empty_and_errors():
    nd = _nd()
    import torch
    res = nd.decompose_batch([], 3, 4)
    assert res.rcliques.shape[0] == 0 and len(res.row_offsets) == 1
    good = nd.to_device(inputs.complete_graph(5))
    # vertex id out of its own graph's range (valid only inside the union)
    rp = torch.tensor([0, 1, 2], dtype=torch.int64, device="cuda")
    col = torch.tensor([1, 3], dtype=torch.int32, device="cuda")
    with pytest.raises(nd.NdError) as e:
        nd.decompose_batch([good, (rp, col)], 2, 3)
    assert e.value.name == "ND_EGRAPH"


def test_batch_canonical_rows():
    """options.canonical on a batch: each graph's rows come out in
    lexicographic order (graph-local ids), equal to the oracle's table."""
    nd = _nd()
    gs = mixed_graphs(seed=5, count=24)
    dev = [nd.to_device(g) for g in gs]
    res = nd.decompose_batch(dev, 3, 4, with_counts=True, canonical=True)
    rcl = res.rcliques.cpu().numpy()
    kap = res.kappa.cpu().numpy().view(np.uint32)
    off = res.row_offsets
    for gi, g in enumerate(gs):
        a, b = int(off[gi]), int(off[gi + 1])
        ref = oracle.decompose(g.n, g.row_ptr, g.col, 3, 4)
        np.testing.assert_array_equal(rcl[a:b], ref.rcliques)
        np.testing.assert_array_equal(kap[a:b].astype(np.uint64), ref.kappa)


def test_autotuned_batch():
    """The schedule autotuner times every candidate on a held-out sample and
    returns the fastest; the batch decomposed with it matches the oracle."""
    nd = _nd()
    gs = mixed_graphs(seed=11, count=40)
    dev = [nd.to_device(g) for g in gs]
    best, rep = nd.nd_batch_autotune(dev, 3, 4, sample_count=12)
    assert rep["sample_graphs"] == 12 and len(rep["candidates"]) == 8
    times = [c["ms"] for c in rep["candidates"]]
    assert all(t > 0 for t in times)
    assert rep["candidates"][rep["best"]]["ms"] == min(times)
    for k in ("orient", "queue_depth", "graph_rounds"):
        assert best[k] == rep["candidates"][rep["best"]][k]
    res = nd.decompose_batch(dev, 3, 4, orient=best["orient"], queue_depth=best["queue_depth"],
                             graph_rounds=bool(best["graph_rounds"]))
    rcl = res.rcliques.cpu().numpy()
    kap = res.kappa.cpu().numpy().view(np.uint32)
    off = res.row_offsets
    for gi, g in enumerate(gs):
        a, b = int(off[gi]), int(off[gi + 1])
        ref = oracle.decompose(g.n, g.row_ptr, g.col, 3, 4)
        grc, gk = _canon(rcl[a:b], kap[a:b])
        np.testing.assert_array_equal(grc, ref.rcliques)
        np.testing.assert_array_equal(gk.astype(np.uint64), ref.kappa)
