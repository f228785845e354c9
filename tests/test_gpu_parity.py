"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is exact (all arithmetic is integer): the r-clique table,
initial counts, nucleus numbers, the number of rounds, every round's size
and level, and the total number of decrements.  Rows are compared after a
lexicographic sort (the library's row order is its table order).
"""
import sys
from math import comb

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


def run_gpu(g, r, s, **kw):
    nd = _nd()
    rp, col = nd.to_device(g)
    d = nd.decompose(rp, col, r, s, with_counts=True, **kw)
    rcl = d.rcliques.cpu().numpy()
    kap = d.kappa.cpu().numpy().view(np.uint32)
    cnt = d.counts.cpu().numpy().view(np.uint32)
    return rcl, kap, cnt, d


def check_against_oracle(g, r, s, **kw):
    print(f"[parity] n={g.n} m={g.m} r={r} s={s} {kw}", flush=True)
    rcl, kap, cnt, d = run_gpu(g, r, s, **kw)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    grc, gk, gc = _canon(rcl, kap, cnt)
    assert grc.shape == ref.rcliques.shape
    np.testing.assert_array_equal(grc, ref.rcliques)
    np.testing.assert_array_equal(gc.astype(np.uint64), ref.counts)
    np.testing.assert_array_equal(gk.astype(np.uint64), ref.kappa)
    assert d.stats["n_s"] == ref.n_s
    assert d.stats["n_r"] == ref.n_r
    assert d.stats["rounds"] == ref.rounds
    np.testing.assert_array_equal(d.round_sizes, ref.round_sizes)
    np.testing.assert_array_equal(d.round_levels.astype(np.uint64), ref.round_k)
    assert d.stats["decrements"] == ref.decrements
    # a decrement of a count already at the level needs no atomic; the first
    # decrement of any count in a round always does
    assert d.stats["atomics"] <= d.stats["decrements"]
    assert (d.stats["atomics"] > 0) == (d.stats["decrements"] > 0)
    return d


RS_ALL = [(1, 2), (1, 3), (2, 3), (2, 4), (3, 4), (3, 5), (4, 5), (2, 5), (1, 4), (4, 6),
          (5, 6), (3, 6), (2, 6), (1, 5), (5, 7), (6, 7), (1, 6), (2, 7)]


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("r,s", [(3, 4), (2, 3), (1, 2), (4, 5), (2, 4), (1, 3)])
def test_worked_example(r, s, generic):
    check_against_oracle(inputs.worked_example(), r, s, generic=generic)


@pytest.mark.parametrize("r,s", RS_ALL)
def test_planted_small_all_rs(r, s):
    g = inputs.planted_er(120, 6.0, 3, 6, 11, 31)
    d = check_against_oracle(g, r, s)
    assert d.stats["key_words"] == 1


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6, 7])
def test_s_equals_8(r):
    """s = 8 (ND_MAX_S) for every r: planted cliques of 9-12 vertices hold
    8-cliques; (7,8) keys need 6 * ceil(log2 n) <= 63, so n <= 1024."""
    g = inputs.planted_er(110, 5.0, 3, 9, 12, 80 + r)
    check_against_oracle(g, r, 8)


@pytest.mark.parametrize("contract", [False, True])
@pytest.mark.parametrize("g", ["rmat12", "rmat_paper11", "planted", "er"])
def test_23_graph_contraction(g, contract):
    """(2,3) with and without graph contraction (Section 4.6): the listed
    adjacency of vertices that lost a quarter of their neighbours is filtered
    of peeled edges after every 2n peeled edges; results stay exact and the
    contraction passes happen when enough edges are peeled."""
    graph = {"rmat12": lambda: inputs.rmat(12, 16, 71),
             "rmat_paper11": lambda: inputs.rmat_paper(11, 24, 72),
             "planted": lambda: inputs.planted_er(1500, 12.0, 6, 10, 40, 73),
             "er": lambda: inputs.erdos_renyi(800, 12000, 74)}[g]()
    d = check_against_oracle(graph, 2, 3, contract=contract)
    if not contract:
        assert d.stats["contractions"] == 0
    elif d.stats["n_r"] >= 4 * graph.n:
        assert d.stats["contractions"] > 0
    # every triangle is listed once, by the edge that owns it
    assert d.stats["discoveries"] == d.stats["n_s"]


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (4, 5), (5, 6), (6, 7)])
def test_generic_path_for_s_eq_r_plus_1(r, s):
    """The generic path (Count-Func atomics, intersection by edge tests) on
    the shapes the bitmap/apex-list path normally serves."""
    g = inputs.planted_er(150, 7.0, 3, 7, 12, 41)
    check_against_oracle(g, r, s, generic=True)


def heavy_root_graph(seed=12):
    """Vertex 0 adjacent to A = {1..600}; every a in A also has 601 private
    leaves, so in degree order 0 ranks below all of A and has 600 > 512
    out-neighbours (no bitmap).  A sparse random graph plus planted cliques
    inside A gives 0 many triangles, 4-cliques and 5-cliques."""
    import numpy as np
    rng = np.random.default_rng(seed)
    k, leaves = 600, 601
    us, vs = [np.zeros(k, dtype=np.int64)], [np.arange(1, k + 1, dtype=np.int64)]
    leaf0 = k + 1
    a = np.repeat(np.arange(1, k + 1, dtype=np.int64), leaves)
    us.append(a)
    vs.append(leaf0 + np.arange(k * leaves, dtype=np.int64))
    inner = inputs.erdos_renyi(k, 2400, seed)
    iu, iv = inputs.edges_of(inner)
    us.append(iu + 1)
    vs.append(iv + 1)
    for _ in range(6):
        c = rng.choice(k, size=int(rng.integers(6, 11)), replace=False) + 1
        x, y = np.triu_indices(len(c), 1)
        us.append(c[x])
        vs.append(c[y])
    n = leaf0 + k * leaves
    return inputs.csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (4, 5)])
def test_heavy_root_fallback_in_fast_path(r, s):
    """Roots with more than 512 out-neighbours keep no bitmap; the s = r+1
    path then tests x > v1 with edge tests."""
    d = check_against_oracle(heavy_root_graph(), r, s)
    assert d.stats["max_out_degree"] > 512


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (2, 4), (1, 2), (4, 5)])
def test_er_medium(seed, r, s):
    g = inputs.erdos_renyi(1500, 15000 if s - r == 1 else 9000, seed)
    check_against_oracle(g, r, s)


def test_er_2000_23_full_workload():
    """The (2,3) workload at its full size: G(n=2,000, m=10,000)."""
    for seed in (1, 2, 3, 4, 5):
        check_against_oracle(inputs.er_2000(seed), 2, 3)


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("r,s", [(3, 4), (2, 3), (2, 4), (1, 2), (4, 5), (1, 3)])
def test_rmat_small(r, s, generic):
    g = inputs.rmat(10, 8, 123)
    check_against_oracle(g, r, s, generic=generic)


@pytest.mark.parametrize("r,s", [(1, 3), (2, 4), (3, 5), (1, 4), (2, 5), (3, 6)])
def test_rmat_flattened_update(r, s):
    """s >= r+2 peels through the flattened candidate / out-arc passes; hub
    r-cliques with large common neighbourhoods are shared across waves."""
    g = inputs.rmat(11, 8, 77)
    check_against_oracle(g, r, s)


@pytest.mark.parametrize("ef", [2, 4, 8, 16])
@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (4, 5)])
def test_paper_rmat_density_sweep_small(ef, r, s):
    """The paper's own rMAT parameters (a=.5, b=c=.1, d=.3) over a density
    sweep, at a size the oracle finishes quickly."""
    check_against_oracle(inputs.rmat_paper(9, ef, 5000 + ef), r, s)


@pytest.mark.parametrize("r,s", [(3, 4), (4, 5), (2, 4)])
def test_chung_lu_small(r, s):
    g = inputs.chung_lu_planted(3000, 8.0, 2.1, 4, 8, 16, 77)
    check_against_oracle(g, r, s)


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4)])
def test_core_order_orientation(r, s):
    g = inputs.rmat(10, 8, 9)
    check_against_oracle(g, r, s, orient=1)


@pytest.mark.parametrize("lf", [0.25, 0.9])
def test_load_factors(lf):
    g = inputs.planted_er(200, 8.0, 2, 8, 14, 5)
    check_against_oracle(g, 3, 4, load_factor=lf)


@pytest.mark.parametrize("n,r,s", [(8, 3, 4), (40, 2, 3), (70, 1, 3), (65, 2, 4), (129, 1, 2),
                                   (260, 1, 2), (300, 2, 3), (520, 1, 2), (600, 1, 3),
                                   (530, 2, 3)])
def test_complete_graph_closed_form(n, r, s):
    """K_n: every r-clique in C(n-r, s-r) s-cliques, all peeled in one round.
    n > 513 sends roots through the heavy-root kernel."""
    print(f"[parity] K_{n} r={r} s={s}", flush=True)
    rcl, kap, cnt, d = run_gpu(inputs.complete_graph(n), r, s)
    assert rcl.shape[0] == comb(n, r)
    assert (cnt == comb(n - r, s - r)).all()
    assert (kap == comb(n - r, s - r)).all()
    assert d.stats["n_s"] == comb(n, s)
    assert d.stats["rounds"] == 1


def test_disjoint_cliques():
    sizes = [3, 5, 9, 17, 33, 65, 70]
    g = inputs.disjoint_union([inputs.complete_graph(k) for k in sizes])
    check_against_oracle(g, 2, 3)
    check_against_oracle(g, 3, 4)


def _tree(arity, depth):
    """Complete arity-ary tree: internal vertices have degree arity + 1."""
    u, v, nxt, level = [], [], 1, [0]
    for _ in range(depth):
        new = []
        for p in level:
            for _ in range(arity):
                u.append(p)
                v.append(nxt)
                new.append(nxt)
                nxt += 1
        level = new
    return inputs.csr_from_edges(nxt, np.array(u), np.array(v))


@pytest.mark.parametrize("generic", [False, True])
def test_window_of_peeled_entries_dropped(generic):
    """(1,2) on a 9-ary tree beside K_21: the first level advance puts the
    tree's internal vertices (degree 10) in the level window and K_21
    (degree 20) above it; all of the tree peels at level 1, so the next
    advance finds a window list that holds only peeled entries and must drop
    it (an empty round, not counted) before it reaches the clique's level."""
    g = inputs.disjoint_union([_tree(9, 3), inputs.complete_graph(21)])
    d = check_against_oracle(g, 1, 2, generic=generic)
    assert list(np.unique(d.round_levels)) == [1, 20]


def test_empty_and_isolated():
    nd = _nd()
    g = inputs.csr_from_edges(10, [], [])
    rcl, kap, cnt, d = run_gpu(g, 1, 2)
    assert rcl.shape == (10, 1) and (kap == 0).all() and d.stats["rounds"] == 1
    rcl, kap, cnt, d = run_gpu(g, 2, 3)
    assert rcl.shape == (0, 2) and d.stats["rounds"] == 0
    # a single edge plus isolated vertices
    g = inputs.csr_from_edges(6, [1], [4])
    check_against_oracle(g, 1, 2)
    check_against_oracle(g, 2, 3)


def test_determinism():
    g = inputs.rmat(11, 8, 4)
    a = run_gpu(g, 3, 4)
    b = run_gpu(g, 3, 4)
    ca, cb = _canon(a[0], a[1], a[2]), _canon(b[0], b[1], b[2])
    for x, y in zip(ca, cb):
        np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------------ errors

def _raw(n, rows):
    import torch
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(x) for x in rows])
    col = np.array([c for x in rows for c in x] or [0], dtype=np.int32)[: rp[-1]]
    return torch.from_numpy(rp).cuda(), torch.from_numpy(col.copy()).cuda()


@pytest.mark.parametrize("rows", [[[1, 1], [0]], [[0], []], [[1], []], [[2, 1], [0], [0]],
                                  [[5], []], [[-1], []]])
def test_malformed_graph_rejected(rows):
    nd = _nd()
    rp, col = _raw(len(rows), rows)
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 2, 3)
    assert e.value.name == "ND_EGRAPH"


def test_bad_arguments():
    nd = _nd()
    rp, col = nd.to_device(inputs.complete_graph(5))
    for r, s in [(0, 2), (2, 2), (3, 1), (1, 9), (8, 9)]:
        with pytest.raises(nd.NdError) as e:
            nd.decompose(rp, col, r, s)
        assert e.value.name == "ND_EINVAL"
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 2, 3, load_factor=0.95)
    assert e.value.name == "ND_EINVAL"
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 2, 3, queue_depth=33)
    assert e.value.name == "ND_EINVAL"


def test_key_width_rejected():
    """Six 22-bit fields (r = 7, n > 2^21) need 132 bits: more than two words."""
    nd = _nd()
    g = inputs.csr_from_edges((1 << 21) + 2, [0, 1], [1, 2])
    rp, col = nd.to_device(g)
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 7, 8)
    assert e.value.name == "ND_EKEYWIDTH"


_WIDE = {}


def _wide_graph(n):
    if n not in _WIDE:
        _WIDE.clear()
        _WIDE[n] = inputs.sparse_with_dense_block(n, 2.0, 200, 0.3, 8, 8, 14, n % 1000)
    return _WIDE[n]


@pytest.mark.parametrize("n,r,s,kw", [
    # n > 2^21: 22-bit fields; r = 4 keys take 66 bits, r = 6 keys 110
    ((1 << 21) + 4096, 4, 5, {}),
    ((1 << 21) + 4096, 4, 5, {"generic": True}),
    ((1 << 21) + 4096, 4, 6, {}),
    ((1 << 21) + 4096, 5, 6, {}),
    ((1 << 21) + 4096, 5, 7, {}),
    ((1 << 21) + 4096, 6, 7, {}),
    # 18-bit fields: r = 7 keys take 108 bits
    ((1 << 17) + 100, 7, 8, {}),
    ((1 << 17) + 100, 5, 6, {"load_factor": 0.9}),
])
def test_two_word_keys(n, r, s, kw):
    """Keys of (r-1) vertex fields wider than 63 bits take a second word.  The
    dense block's vertices get the top ranks (the highest degrees), so their
    fields straddle the two words and fill the second."""
    d = check_against_oracle(_wide_graph(n), r, s, **kw)
    assert d.stats["key_words"] == 2
    assert d.stats["n_s"] > 0


@pytest.mark.parametrize("r,s,kw", [
    (4, 5, {}), (4, 6, {}), (5, 6, {}), (5, 7, {}), (6, 7, {}), (4, 7, {}), (7, 8, {}),
    (4, 5, {"generic": True}), (5, 6, {"generic": True}), (4, 5, {"load_factor": 0.9}),
])
def test_three_level_table(r, s, kw):
    """Three-level r-clique tables (Section 4.1, l = 3): the out-arc (v1, v2)
    selects the last-level table; results identical to the oracle's."""
    g = inputs.sparse_with_dense_block(400, 3.0, 120, 0.35, 10, 8, 13, 77)
    d = check_against_oracle(g, r, s, levels=3, **kw)
    assert d.stats["n_s"] > 0


@pytest.mark.parametrize("n,r,s,words", [
    ((1 << 21) + 4096, 4, 5, 1),  # v3, v4: 44 bits (66 with two levels)
    ((1 << 21) + 4096, 4, 6, 1),
    ((1 << 21) + 4096, 5, 7, 2),  # v3..v5: 66 bits
    ((1 << 21) + 4096, 6, 7, 2),  # v3..v6: 88 bits
])
def test_three_level_key_width(n, r, s, words):
    """With three levels a key carries r-2 vertices, so n > 2^21 keeps (4,*)
    keys in one word."""
    d = check_against_oracle(_wide_graph(n), r, s, levels=3)
    assert d.stats["key_words"] == words


def test_three_level_rejected_below_r4():
    nd = _nd()
    rp, col = nd.to_device(inputs.planted_er(60, 5.0, 2, 5, 8, 3))
    for r, s, lv in [(3, 4, 3), (2, 4, 3), (4, 5, 1), (4, 5, 4)]:
        with pytest.raises(nd.NdError) as e:
            nd.decompose(rp, col, r, s, levels=lv)
        assert e.value.name == "ND_EINVAL"


def test_budget_rejected():
    """A budget below what the plan and its run's workspace need fails at plan
    creation, once n_r is known and before the table is allocated."""
    nd = _nd()
    rp, col = nd.to_device(inputs.rmat(10, 8, 3))
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 3, 4, hbm_budget_bytes=4096)
    assert e.value.name == "ND_ENOMEM"
    plan = nd.nd_plan_create(rp, col, 3, 4)
    _, ws, held = nd.nd_plan_sizes(plan)
    nd.nd_plan_destroy(plan)
    # just below the plan + workspace need: refused; at the need: accepted
    with pytest.raises(nd.NdError) as e:
        nd.nd_plan_create(rp, col, 3, 4, hbm_budget_bytes=held + ws - 1)
    assert e.value.name == "ND_ENOMEM"
    plan = nd.nd_plan_create(rp, col, 3, 4, hbm_budget_bytes=held + ws)
    nd.nd_plan_destroy(plan)


def test_workspace_too_small_rejected_before_any_kernel():
    """nd_run refuses a workspace below nd_plan_sizes' figure with ND_ENOMEM
    and leaves the outputs untouched (no kernel ran)."""
    nd = _nd()
    import torch
    g = inputs.rmat(9, 8, 4)
    rp, col = nd.to_device(g)
    plan = nd.nd_plan_create(rp, col, 3, 4)
    try:
        n_r, ws_bytes, _ = nd.nd_plan_sizes(plan)
        rcl = torch.full((n_r, 3), -7, dtype=torch.int32, device="cuda")
        kap = torch.full((n_r,), -7, dtype=torch.int32, device="cuda")
        ws = nd.workspace(ws_bytes)
        with pytest.raises(nd.NdError) as e:
            nd.nd_run(plan, ws, rcl, kap, ws_bytes=ws_bytes - 1)
        assert e.value.name == "ND_ENOMEM"
        torch.cuda.synchronize()
        assert int((rcl != -7).sum()) == 0 and int((kap != -7).sum()) == 0
        st = nd.nd_run(plan, ws, rcl, kap, ws_bytes=ws_bytes)
        assert st["workspace_bytes"] == ws_bytes  # the reported size is what a run carves
    finally:
        nd.nd_plan_destroy(plan)


def test_plan_lifecycle():
    nd = _nd()
    import torch
    rp, col = nd.to_device(inputs.worked_example())
    plan = nd.nd_plan_create(rp, col, 3, 4)
    n_r, ws_bytes, held = nd.nd_plan_sizes(plan)
    assert n_r == 14 and ws_bytes > 0 and held > 0
    with pytest.raises(nd.NdError) as e:
        nd.nd_round_trace(plan)
    assert e.value.name == "ND_ESTATE"
    rcl = torch.empty((n_r, 3), dtype=torch.int32, device="cuda")
    kap = torch.empty((n_r,), dtype=torch.int32, device="cuda")
    ws = nd.workspace(ws_bytes)
    nd.nd_run(plan, ws, rcl, kap)
    first = (rcl.cpu().numpy().copy(), kap.cpu().numpy().copy())
    sizes, levels = nd.nd_round_trace(plan)
    assert sizes.tolist() == [1, 3, 10] and levels.tolist() == [0, 1, 2]
    # a plan runs again from its table and gives the same result
    rcl.fill_(-1)
    kap.fill_(-1)
    nd.nd_run(plan, ws, rcl, kap)
    assert np.array_equal(rcl.cpu().numpy(), first[0])
    assert np.array_equal(kap.cpu().numpy(), first[1])
    sizes, levels = nd.nd_round_trace(plan)
    assert sizes.tolist() == [1, 3, 10] and levels.tolist() == [0, 1, 2]
    nd.nd_plan_destroy(plan)
    nd.nd_release_cached()


@pytest.mark.parametrize("r,s", [(3, 4), (2, 4), (1, 3), (2, 3), (3, 5)])
def test_round_capacity_requery(r, s):
    """Tiny record / out-arc / round-trace capacities: a round that outgrows
    the workspace stops the run with ND_ENOMEM and the plan reports a larger
    workspace; the run repeated with it is exact."""
    nd = _nd()
    import torch
    g = inputs.rmat(10, 8, 321)
    rp, col = nd.to_device(g)
    plan = nd.nd_plan_create(rp, col, r, s, record_cap=64, trace_cap=2)
    try:
        n_r, ws0, _ = nd.nd_plan_sizes(plan)
        rcl = torch.empty((n_r, r), dtype=torch.int32, device="cuda")
        kap = torch.empty((n_r,), dtype=torch.int32, device="cuda")
        with pytest.raises(nd.NdError) as e:
            nd.nd_run(plan, nd.workspace(ws0), rcl, kap)
        assert e.value.name == "ND_ENOMEM"
        assert nd.nd_plan_sizes(plan)[1] > ws0
    finally:
        nd.nd_plan_destroy(plan)
    check_against_oracle(g, r, s, record_cap=64, trace_cap=2)


@pytest.mark.parametrize("r,s,kw", [
    (3, 4, {}), (2, 4, {}), (2, 3, {"contract": True}), (3, 5, {}), (1, 3, {}), (4, 5, {}),
    (2, 5, {}), (3, 4, {"canonical": True}), (2, 4, {"canonical": True}),
    (3, 4, {"with_counts": False}),
])
def test_round_capacity_resume(r, s, kw):
    """A round that outgrows the records or out-arcs of the workspace stops
    the run with ND_ENOMEM; the next run on the plan, with the workspace it
    then reports, goes on from that round.  Over many such stops the whole
    peel is exact (rows, initial counts, kappa, every round's size and
    level, decrements), and the finishing run does no counting."""
    nd = _nd()
    import torch
    kw = dict(kw)
    with_counts = kw.pop("with_counts", True)
    canonical = kw.get("canonical", False)
    g = inputs.rmat(10, 8, 321)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    rp, col = nd.to_device(g)
    plan = nd.nd_plan_create(rp, col, r, s, record_cap=64, timing=True, **kw)
    try:
        n_r = nd.nd_plan_sizes(plan)[0]
        rcl = torch.empty((n_r, r), dtype=torch.int32, device="cuda")
        kap = torch.empty((n_r,), dtype=torch.int32, device="cuda")
        cnt = torch.empty((n_r,), dtype=torch.int32, device="cuda") if with_counts else None
        stops = 0
        while True:
            ws_bytes = nd.nd_plan_sizes(plan)[1]
            try:
                st = nd.nd_run(plan, nd.workspace(ws_bytes), rcl, kap, cnt, ws_bytes=ws_bytes)
                break
            except nd.NdError as e:
                assert e.name == "ND_ENOMEM"
                stops += 1
                assert stops < 40
        assert stops >= 1
        assert st["count_launches"] == 0  # resumed: the count ran in the first run only
        sizes, levels = nd.nd_round_trace(plan)
    finally:
        nd.nd_plan_destroy(plan)
    rows = rcl.cpu().numpy()
    k = kap.cpu().numpy().view(np.uint32).astype(np.uint64)
    c = cnt.cpu().numpy().view(np.uint32).astype(np.uint64) if with_counts else None
    if canonical:
        np.testing.assert_array_equal(rows, ref.rcliques)
    else:
        order = np.lexsort(rows.T[::-1])
        rows, k = rows[order], k[order]
        c = c[order] if with_counts else None
        np.testing.assert_array_equal(rows, ref.rcliques)
    np.testing.assert_array_equal(k, ref.kappa)
    if with_counts:
        np.testing.assert_array_equal(c, ref.counts)
    np.testing.assert_array_equal(sizes, ref.round_sizes)
    np.testing.assert_array_equal(levels.astype(np.uint64), ref.round_k)
    assert st["rounds"] == ref.rounds
    assert st["n_s"] == ref.n_s
    assert st["decrements"] == ref.decrements


def test_resume_then_fresh_run():
    """After a resumed peel the plan runs again from its table (no stale
    state), and a run asking for counts the stopped run did not take starts
    again instead of resuming."""
    nd = _nd()
    import torch
    g = inputs.rmat(9, 8, 5)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, 3, 4)
    rp, col = nd.to_device(g)
    plan = nd.nd_plan_create(rp, col, 3, 4, record_cap=64)
    try:
        n_r = nd.nd_plan_sizes(plan)[0]
        rcl = torch.empty((n_r, 3), dtype=torch.int32, device="cuda")
        kap = torch.empty((n_r,), dtype=torch.int32, device="cuda")
        cnt = torch.empty((n_r,), dtype=torch.int32, device="cuda")
        ws0 = nd.nd_plan_sizes(plan)[1]
        with pytest.raises(nd.NdError):
            nd.nd_run(plan, nd.workspace(ws0), rcl, kap)  # stops without counts
        for _ in range(40):  # counts now: starts again, then resumes as it stops
            ws_bytes = nd.nd_plan_sizes(plan)[1]
            try:
                nd.nd_run(plan, nd.workspace(ws_bytes), rcl, kap, cnt, ws_bytes=ws_bytes)
                break
            except nd.NdError as e:
                assert e.name == "ND_ENOMEM"
        first = (rcl.cpu().numpy().copy(), kap.cpu().numpy().copy(), cnt.cpu().numpy().copy())
        ws_bytes = nd.nd_plan_sizes(plan)[1]
        st = nd.nd_run(plan, nd.workspace(ws_bytes), rcl, kap, cnt, ws_bytes=ws_bytes)
        assert st["rounds"] == ref.rounds
        for a, b in zip(first, (rcl.cpu().numpy(), kap.cpu().numpy(), cnt.cpu().numpy())):
            assert np.array_equal(a, b)
    finally:
        nd.nd_plan_destroy(plan)
    order = np.lexsort(first[0].T[::-1])
    np.testing.assert_array_equal(first[0][order], ref.rcliques)
    np.testing.assert_array_equal(first[1].view(np.uint32)[order].astype(np.uint64), ref.kappa)
    np.testing.assert_array_equal(first[2].view(np.uint32)[order].astype(np.uint64), ref.counts)


@pytest.mark.parametrize("r,s", [(3, 4), (2, 3), (2, 4), (4, 5), (1, 2)])
def test_canonical_rows(r, s):
    """options.canonical: rows come out in lexicographic order, equal to the
    oracle's table row for row with no host-side sort."""
    g = inputs.planted_er(300, 8.0, 3, 6, 12, 77)
    rcl, kap, cnt, d = run_gpu(g, r, s, canonical=True)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    np.testing.assert_array_equal(rcl, ref.rcliques)
    np.testing.assert_array_equal(cnt.astype(np.uint64), ref.counts)
    np.testing.assert_array_equal(kap.astype(np.uint64), ref.kappa)


def test_canonical_two_keys():
    """r vertices wider than 64 bits (r = 4, n > 2^16 ids): the canonical
    sort runs on two keys."""
    base = inputs.planted_er(400, 6.0, 3, 7, 12, 5)
    g, _ = inputs.permute(inputs.disjoint_union([base, inputs.erdos_renyi(70000, 1000, 6)]), 8)
    rcl, kap, cnt, d = run_gpu(g, 4, 5, canonical=True)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, 4, 5)
    np.testing.assert_array_equal(rcl, ref.rcliques)
    np.testing.assert_array_equal(kap.astype(np.uint64), ref.kappa)


def test_count_bias_overflow():
    """options.debug_count_bias drives the 32-bit range check of the initial
    counts: a bias that lifts the largest count past UINT32_MAX gives
    ND_EOVERFLOW, one that reaches it exactly does not (and changes nothing)."""
    nd = _nd()
    g = inputs.planted_er(200, 6.0, 2, 8, 12, 9)
    ref = oracle.decompose(g.n, g.row_ptr, g.col, 3, 4)
    top = int(ref.counts.max())
    rp, col = nd.to_device(g)
    with pytest.raises(nd.NdError) as e:
        nd.decompose(rp, col, 3, 4, debug_count_bias=(1 << 32) - top)
    assert e.value.name == "ND_EOVERFLOW"
    check_against_oracle(g, 3, 4, debug_count_bias=(1 << 32) - 1 - top)
    with pytest.raises(nd.NdError) as e:  # the generic (Count-Func atomics) path too
        nd.decompose(rp, col, 3, 4, generic=True, debug_count_bias=(1 << 32) - top)
    assert e.value.name == "ND_EOVERFLOW"


@pytest.mark.parametrize("depth", [1, 4])
def test_round_queue_depth(depth):
    """Results do not depend on how many rounds are queued between reads of
    the device round state."""
    check_against_oracle(inputs.rmat(10, 8, 55), 2, 4, queue_depth=depth)


@pytest.mark.parametrize("r,s", [(3, 4), (2, 4), (2, 3), (4, 5), (1, 2), (3, 5)])
@pytest.mark.parametrize("timing", [False, True])  # timed runs fall back to plain launches
def test_graph_replayed_rounds(r, s, timing):
    """options.graph_rounds: the rounds queued after the first of every batch
    run from captured HIP graphs, each replayed many times within the peel
    (with the host's reads of the round state between replays); every round
    and the final result equal the oracle's."""
    g = inputs.rmat(10, 10, 300 + r)
    d = check_against_oracle(g, r, s, graph_rounds=True, timing=timing, queue_depth=4)
    assert d.stats["rounds"] > 12  # several batches of 4, so graphs are replayed


def _random_case(seed):
    rng = np.random.default_rng(seed)
    kind = int(rng.integers(0, 5))
    sd = int(rng.integers(0, 2**31))
    if kind == 0:
        n = int(rng.integers(2, 120))
        g = inputs.erdos_renyi(n, int(rng.integers(0, min(n * (n - 1) // 2, 6 * n) + 1)), sd)
    elif kind == 1:
        g = inputs.planted_er(int(rng.integers(20, 200)), float(rng.uniform(1, 10)),
                              int(rng.integers(1, 5)), 4, 14, sd)
    elif kind == 2:
        g = inputs.rmat(int(rng.integers(4, 10)), int(rng.integers(2, 17)), sd)
    elif kind == 3:
        g = inputs.rmat_paper(int(rng.integers(4, 10)), int(rng.integers(2, 17)), sd)
    else:
        g = inputs.disjoint_union([inputs.complete_graph(int(k))
                                   for k in rng.integers(1, 12, size=int(rng.integers(1, 6)))])
    r = int(rng.integers(1, 6))
    s = r + int(rng.integers(1, min(3, 7 - r) + 1))
    return g, r, s


@pytest.mark.parametrize("seed", range(40))
def test_random_graphs_and_rs(seed):
    """Seeded random graphs of every generator and random (r, s), s <= r+3."""
    g, r, s = _random_case(9000 + seed)
    check_against_oracle(g, r, s)
