"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: the values the paper
prints for its worked example (tests/golden), brute force straight from the
definition on tiny graphs, closed forms (complete graphs and disjoint unions),
the count identity, the k-core / k-truss special cases through networkx, an
independent local (h-index) algorithm, a round-by-round recount and
invariance under vertex relabeling.
"""
import json
import os
from itertools import combinations
from math import comb

import networkx as nx
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import oracle
from paper_2111_10980_amd import inputs
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RS_SMALL = [(1, 2), (1, 3), (2, 3), (2, 4), (3, 4), (3, 5), (4, 5), (2, 5), (1, 4)]


def _names(rows):
    return ["".join(inputs.EXAMPLE_NAMES[x] for x in row) for row in rows]


# --------------------------------------------------------------- worked example

def test_worked_example_matches_printed_values():
    fx = json.load(open(os.path.join(GOLDEN, "worked_example_34.json")))
    g = inputs.worked_example()
    # the fixture's edge list and the generator's agree
    edges = sorted("".join(sorted(e)) for e in fx["graph"]["edges"])
    u, v = inputs.edges_of(g)
    assert sorted(_names(zip(u, v))) == edges
    res = oracle.decompose(g.n, g.row_ptr, g.col, fx["r"], fx["s"])
    names = _names(res.rcliques)
    assert res.n_r == fx["n_triangles"]
    assert dict(zip(names, res.counts.tolist())) == fx["initial_counts"]
    assert dict(zip(names, res.kappa.tolist())) == fx["kappa"]
    assert res.rounds == fx["rounds"]
    assert np.cumsum(res.round_sizes).tolist() == fx["finished_after_round"]
    assert res.round_k.tolist() == fx["round_level"]
    changed = [nm for nm, a, b in zip(names, res.counts, res.final_counts) if a != b]
    assert changed == fx["updated_in_round_2"]
    assert int(res.final_counts[names.index("abe")]) == fx["count_of_abe_after_round_2"]
    # the single-removal peel agrees on kappa
    single = oracle.decompose(g.n, g.row_ptr, g.col, 3, 4, single=True)
    assert single.kappa.tolist() == res.kappa.tolist()


@pytest.mark.parametrize("r,s", [(1, 2), (1, 3), (2, 3), (2, 4), (4, 5), (3, 5)])
def test_worked_example_other_rs_by_brute_force(r, s):
    g = inputs.worked_example()
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    Kr, kap = brute.kappa_by_subsets(g.n, g.row_ptr, g.col, r, s) if comb(7, r) <= 16 and r >= 3 \
        else brute.kappa_by_cores(g.n, g.row_ptr, g.col, r, s)
    assert brute.rows_dict(res.rcliques, res.kappa) == brute.as_dict(Kr, kap)


def test_worked_example_known_cases():
    """(4,5): abef is in no 5-clique; the five 4-cliques of the 5-clique
    have kappa 1.  (1,2): k-core; (2,3): k-truss."""
    g = inputs.worked_example()
    res = oracle.decompose(g.n, g.row_ptr, g.col, 4, 5)
    d = dict(zip(_names(res.rcliques), res.kappa.tolist()))
    assert d == {"abcd": 1, "abce": 1, "abde": 1, "abef": 0, "acde": 1, "bcde": 1}
    assert res.rounds == 2
    res = oracle.decompose(g.n, g.row_ptr, g.col, 1, 2)
    assert res.kappa.tolist() == [4, 4, 4, 4, 4, 3, 2]


# ------------------------------------------------------------- brute force

def _graph_from_mask(n, mask_bits):
    pairs = list(combinations(range(n), 2))
    e = [p for p, b in zip(pairs, mask_bits) if b]
    if not e:
        return inputs.csr_from_edges(n, [], [])
    a = np.array(e, dtype=np.int64)
    return inputs.csr_from_edges(n, a[:, 0], a[:, 1])


@st.composite
def tiny_graphs(draw, nmax=9):
    n = draw(st.integers(min_value=1, max_value=nmax))
    p = draw(st.sampled_from([0.3, 0.5, 0.7, 0.9]))
    bits = draw(st.lists(st.floats(min_value=0, max_value=1), min_size=n * (n - 1) // 2,
                         max_size=n * (n - 1) // 2))
    return _graph_from_mask(n, [b < p for b in bits])


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=tiny_graphs(), rs=st.sampled_from(RS_SMALL))
def test_kappa_matches_core_definition(g, rs):
    r, s = rs
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    Kr, kap = brute.kappa_by_cores(g.n, g.row_ptr, g.col, r, s)
    assert brute.rows_dict(res.rcliques, res.kappa) == brute.as_dict(Kr, kap)
    Kr2, cnt = brute.counts(g.n, g.row_ptr, g.col, r, s)
    assert brute.rows_dict(res.rcliques, res.counts) == brute.as_dict(Kr2, cnt)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=tiny_graphs(nmax=7), rs=st.sampled_from([(1, 2), (2, 3), (1, 3), (2, 4), (3, 4)]))
def test_kappa_matches_subset_enumeration(g, rs):
    r, s = rs
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    if res.n_r > 14:
        return
    Kr, kap = brute.kappa_by_subsets(g.n, g.row_ptr, g.col, r, s)
    assert brute.rows_dict(res.rcliques, res.kappa) == brute.as_dict(Kr, kap)


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=tiny_graphs(nmax=10), rs=st.sampled_from(RS_SMALL))
def test_rounds_match_recount(g, rs):
    """Round count, round sizes and levels of the bulk peel equal a simulation
    that recomputes every count from scratch each round."""
    r, s = rs
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    Kr, kap, sizes, levels = brute.rounds_by_recount(g.n, g.row_ptr, g.col, r, s)
    assert res.rounds == len(sizes)
    assert res.round_sizes.tolist() == sizes
    assert res.round_k.tolist() == levels
    assert brute.rows_dict(res.rcliques, res.kappa) == brute.as_dict(Kr, kap)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=tiny_graphs(nmax=11), rs=st.sampled_from(RS_SMALL))
def test_hindex_local_algorithm_agrees(g, rs):
    r, s = rs
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    Kr, tau = brute.kappa_by_hindex(g.n, g.row_ptr, g.col, r, s)
    assert brute.rows_dict(res.rcliques, res.kappa) == brute.as_dict(Kr, tau)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 2, 5, 8, 12])
@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4), (2, 5), (4, 6), (1, 5), (5, 7)])
def test_complete_graph_closed_form(n, r, s):
    g = inputs.complete_graph(n)
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    assert res.n_r == comb(n, r)
    assert res.n_s == comb(n, s)
    expect = comb(n - r, s - r) if n >= r else 0
    assert (res.counts == expect).all()
    assert (res.kappa == expect).all()
    assert res.rounds == (1 if res.n_r else 0)


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4), (2, 4), (3, 5)])
def test_disjoint_cliques(r, s):
    sizes = [3, 4, 6, 7, 9]
    g = inputs.disjoint_union([inputs.complete_graph(k) for k in sizes])
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    off = np.cumsum([0] + sizes)
    comp = np.searchsorted(off, res.rcliques[:, 0], side="right") - 1
    for c, k in enumerate(sizes):
        sel = comp == c
        assert sel.sum() == comb(k, r)
        assert (res.kappa[sel] == comb(k - r, s - r)).all()
    # rounds: one per distinct level present
    assert res.rounds == len({comb(k - r, s - r) for k in sizes if k >= r})


# --------------------------------------------------------------- identities

@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4), (2, 4), (1, 3), (3, 5)])
def test_count_identity_and_bounds(seed, r, s):
    g = inputs.erdos_renyi(60, 500, seed)
    res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    assert int(res.counts.sum()) == comb(s, r) * res.n_s
    assert (res.kappa <= res.counts).all()
    assert res.max_kappa == int(res.kappa.max()) if res.n_r else True
    # every s-clique is destroyed exactly once: each one contributes
    # C(s,r) - a decrements, a >= 1
    assert res.decrements <= (comb(s, r) - 1) * res.n_s
    # every peeled r-clique re-finds all of its s-cliques
    assert res.discoveries == comb(s, r) * res.n_s
    # one-at-a-time peeling gives the same numbers
    single = oracle.decompose(g.n, g.row_ptr, g.col, r, s, single=True)
    assert (single.kappa == res.kappa).all()


def test_certificate_local_conditions():
    """kappa(R) is supported at its own level and not one above (the fixed
    point property the local algorithm converges to)."""
    g = inputs.erdos_renyi(40, 260, 5)
    for r, s in [(2, 3), (3, 4), (1, 3)]:
        res = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
        tab = oracle.KappaTable(g.n, res.rcliques, res.kappa)
        for R, k in zip(res.rcliques, res.kappa):
            k = int(k)
            assert oracle.support_at(g.n, g.row_ptr, g.col, r, s, tab, R, k) >= k
            assert oracle.support_at(g.n, g.row_ptr, g.col, r, s, tab, R, k + 1) <= k


def test_count_one_matches_table():
    g = inputs.erdos_renyi(80, 700, 3)
    res = oracle.count(g.n, g.row_ptr, g.col, 3, 4)
    for R, c in list(zip(res.rcliques, res.counts))[:200]:
        assert oracle.count_one(g.n, g.row_ptr, g.col, 3, 4, R) == int(c)


# ---------------------------------------------------------- k-core / k-truss

def _nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    u, v = inputs.edges_of(g)
    G.add_edges_from(zip(u.tolist(), v.tolist()))
    return G


@pytest.mark.parametrize("gen", ["er", "rmat", "planted"])
def test_kcore_is_nucleus_12(gen):
    g = {"er": lambda: inputs.erdos_renyi(300, 1500, 4),
         "rmat": lambda: inputs.rmat(9, 8, 5),
         "planted": lambda: inputs.planted_er(200, 6.0, 3, 8, 15, 6)}[gen]()
    res = oracle.decompose(g.n, g.row_ptr, g.col, 1, 2)
    core = nx.core_number(_nx_graph(g))
    assert res.kappa.tolist() == [core[v] for v in range(g.n)]


@pytest.mark.parametrize("gen", ["er", "rmat", "planted"])
def test_ktruss_is_nucleus_23(gen):
    g = {"er": lambda: inputs.erdos_renyi(150, 900, 7),
         "rmat": lambda: inputs.rmat(8, 8, 8),
         "planted": lambda: inputs.planted_er(120, 5.0, 3, 6, 12, 9)}[gen]()
    res = oracle.decompose(g.n, g.row_ptr, g.col, 2, 3)
    G = _nx_graph(g)
    kap = brute.rows_dict(res.rcliques, res.kappa)
    # edge e lies in networkx's k-truss  <=>  kappa(e) >= k - 2
    kmax = int(res.kappa.max()) + 3
    for k in range(2, kmax + 1):
        T = nx.k_truss(G, k)
        inside = {tuple(sorted(e)) for e in T.edges()}
        expect = {e for e, c in kap.items() if c >= k - 2}
        assert inside == expect, k


# ------------------------------------------------------------- invariances

@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (1, 3), (2, 4)])
def test_relabeling_invariance(r, s):
    g = inputs.planted_er(150, 7.0, 3, 6, 12, 11)
    h, perm = inputs.permute(g, 99)
    a = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
    b = oracle.decompose(h.n, h.row_ptr, h.col, r, s)
    da = {tuple(sorted(perm[x] for x in R)): int(k) for R, k in zip(a.rcliques, a.kappa)}
    db = brute.rows_dict(b.rcliques, b.kappa)
    assert da == db
    assert a.rounds == b.rounds
    assert a.round_sizes.tolist() == b.round_sizes.tolist()
    assert a.decrements == b.decrements


# ---------------------------------------------------------------- validation

def _raw(n, rows):
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(x) for x in rows])
    col = np.array([c for x in rows for c in x], dtype=np.int32)
    return rp, col


@pytest.mark.parametrize("rows,code", [
    ([[1], [0]], 0),
    ([[1, 1], [0]], 2),          # duplicate
    ([[0], []], 2),              # self-loop
    ([[1], []], 2),              # asymmetric
    ([[2, 1], [0], [0]], 2),     # unsorted
    ([[5], []], 2),              # out of range
])
def test_validation(rows, code):
    rp, col = _raw(len(rows), rows)
    assert oracle.validate(len(rows), rp, col) == code
    if code:
        with pytest.raises(oracle.OracleError):
            oracle.decompose(len(rows), rp, col, 2, 3)


def test_bad_rs():
    g = inputs.complete_graph(4)
    for r, s in [(0, 2), (2, 2), (3, 2), (1, 9)]:
        with pytest.raises(oracle.OracleError):
            oracle.decompose(g.n, g.row_ptr, g.col, r, s)


def test_empty_graphs():
    g = inputs.csr_from_edges(5, [], [])
    res = oracle.decompose(g.n, g.row_ptr, g.col, 1, 2)
    assert res.n_r == 5 and (res.kappa == 0).all() and res.rounds == 1
    res = oracle.decompose(g.n, g.row_ptr, g.col, 2, 3)
    assert res.n_r == 0 and res.rounds == 0
    g0 = inputs.csr_from_edges(0, [], [])
    res = oracle.decompose(0, g0.row_ptr, g0.col, 1, 2)
    assert res.n_r == 0


def test_certificate_excludes_the_rclique_itself():
    """(1,2) on the worked example: vertex g (kappa 2) has two edges whose
    other endpoints c, d have kappa 4, so its support at threshold 3 counts
    both, although g's own kappa is below 3."""
    g = inputs.worked_example()
    res = oracle.decompose(g.n, g.row_ptr, g.col, 1, 2)
    tab = oracle.KappaTable(g.n, res.rcliques, res.kappa)
    assert oracle.support_at(g.n, g.row_ptr, g.col, 1, 2, tab, [6], 3) == 2
    assert oracle.support_at(g.n, g.row_ptr, g.col, 1, 2, tab, [6], 5) == 0
