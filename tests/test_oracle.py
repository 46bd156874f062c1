"""Pins for the CPU oracle (no GPU).

The oracle (Dinic and two-phase FIFO push-relabel in ``oracle/``) is checked
against things other than itself:

* brute-force enumeration of every s-t cut on tiny multigraphs (max-flow
  min-cut theorem, section 2.1 of the paper: the maximum flow value equals
  the minimum cut capacity);
* closed forms (a path carries its minimum capacity; disjoint paths add; a
  complete unit bipartite graph with super-source/sink matches the smaller
  side; a grid whose neighbour links are all zero carries
  sum_p min(c(s,p), c(p,t)); an unreachable sink carries nothing);
* library routines for special cases: scipy's maximum_flow (a different
  implementation of the same definition) and Hopcroft-Karp maximum bipartite
  matching (the matching workload of section 4 reduces to it);
* invariants: feasibility, value == cut capacity, and the canonical sink side
  (vertices that reach t in the residual graph) being identical for two
  different maximum flows;
* the canonical sink side against brute force: among all minimum s-t cuts,
  the set of vertices that reach t in the residual graph of a maximum flow
  is the smallest sink side, i.e. the intersection of the sink sides of
  every minimum cut (Picard-Queyranne); enumerating all cuts of tiny graphs
  gives that intersection without any flow;
* planted mistakes, which the certificate must reject.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import maximum_bipartite_matching, maximum_flow

import oracle
from paper_2404_00270_amd import workloads as W


def solve_both(g):
    a = oracle.dinic(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    b = oracle.fifo_pr(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    return a, b


def certify(g, res):
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, res.flow)
    assert c.feasible, (c.code, c.bad)
    assert c.value == res.value
    assert c.is_maximum(g.s)
    return c


def _all_cut_capacities(g):
    """(S, capacities): every one of the 2^(V-2) s-t cuts as a boolean
    source-side matrix S (one row per cut) and its capacity."""
    V, s, t = g.V, g.s, g.t
    others = [v for v in range(V) if v not in (s, t)]
    k = len(others)
    masks = np.array(list(itertools.product([0, 1], repeat=k)), dtype=bool).reshape(2**k, k)
    S = np.zeros((masks.shape[0], V), dtype=bool)  # True = source side
    S[:, s] = True
    S[:, others] = masks
    src = W.arc_sources(g)
    cut = S[:, src] & ~S[:, g.col]
    caps = cut.astype(np.int64) @ g.cap.astype(np.int64) if g.E else np.zeros(S.shape[0], np.int64)
    return S, caps


def brute_force_min_cut(g):
    """Minimum over all 2^(V-2) s-t cuts of the cut capacity (vectorised)."""
    _, caps = _all_cut_capacities(g)
    return int(caps.min())


def brute_force_sink_side(g):
    """Intersection of the sink sides of all minimum s-t cuts (uint8[V]): the
    sink-nearest minimum cut, found by enumeration without any flow."""
    S, caps = _all_cut_capacities(g)
    T = ~S[caps == caps.min()]
    return np.logical_and.reduce(T, axis=0).astype(np.uint8)


@pytest.mark.parametrize("seed", range(120))
def test_bruteforce_multigraphs(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 12))
    E = int(rng.integers(0, 5 * V))
    g = W.multigraph(V, E, cmax=int(rng.integers(0, 25)), seed=1000 + seed)
    want = brute_force_min_cut(g)
    a, b = solve_both(g)
    assert a.value == want
    assert b.value == want
    ca, cb = certify(g, a), certify(g, b)
    # the sink side of a minimum cut read from the residual graph does not
    # depend on which maximum flow produced it ...
    assert np.array_equal(ca.side, cb.side)
    # ... and is the sink-nearest minimum cut: the intersection of the sink
    # sides of every minimum cut, from enumeration alone
    assert np.array_equal(ca.side, brute_force_sink_side(g))


@pytest.mark.parametrize("seed", range(60))
def test_canonical_side_is_sink_nearest_min_cut(seed):
    """Graphs with many tied minimum cuts (small capacities from {0, 1, 2}),
    so the source-nearest and sink-nearest minimum cuts usually differ and a
    side read the wrong way round (the complement of what s reaches) fails."""
    rng = np.random.default_rng(5000 + seed)
    V = int(rng.integers(3, 11))
    g = W.multigraph(V, int(rng.integers(V, 4 * V)), cmax=2, seed=9000 + seed)
    want = brute_force_sink_side(g)
    for r in solve_both(g):
        c = certify(g, r)
        assert np.array_equal(c.side, want)


def test_canonical_side_hand_cases():
    # path 0 -> 1 -> 2 with equal capacities: both arcs are minimum cuts;
    # only t reaches t in the residual graph, so the side is [0, 0, 1]
    g = W.from_arcs(3, [(0, 1, 5), (1, 2, 5)], 0, 2)
    for r in solve_both(g):
        assert certify(g, r).side.tolist() == [0, 0, 1]
    assert brute_force_sink_side(g).tolist() == [0, 0, 1]
    # a bottleneck in the middle of a longer path: 0 -5-> 1 -2-> 2 -5-> 3;
    # vertices after the bottleneck still reach t, those before it do not
    g = W.from_arcs(4, [(0, 1, 5), (1, 2, 2), (2, 3, 5)], 0, 3)
    for r in solve_both(g):
        assert certify(g, r).side.tolist() == [0, 0, 1, 1]
    # two tied cuts around vertex 1 with a side branch 1 -> 2 -> 3(t): after
    # the maximum flow of 3 on 0 -> 1 -> 3, vertex 2 still reaches t through
    # its own arc, 1 does not (its arcs to 2 and 3 are saturated or absent)
    g = W.from_arcs(4, [(0, 1, 3), (1, 3, 3), (2, 3, 4)], 0, 3)
    for r in solve_both(g):
        assert certify(g, r).side.tolist() == [0, 0, 1, 1]
    assert brute_force_sink_side(g).tolist() == [0, 0, 1, 1]


def _path(caps):
    V = len(caps) + 1
    return W.from_arcs(V, [(i, i + 1, c) for i, c in enumerate(caps)], 0, V - 1)


@pytest.mark.parametrize("caps", [[5], [3, 7, 2, 9], [0, 4], [10, 10, 10], [1] * 50, [2**31 - 1, 2**31 - 1]])
def test_path_is_min_capacity(caps):
    g = _path(caps)
    for r in solve_both(g):
        assert r.value == min(caps)
        certify(g, r)


def test_disjoint_paths_add():
    rng = np.random.default_rng(7)
    arcs, V, want = [], 2, 0
    s, t = 0, 1
    for _ in range(20):
        L = int(rng.integers(1, 6))
        caps = rng.integers(0, 50, size=L + 1).tolist()
        nodes = [s] + list(range(V, V + L)) + [t]
        V += L
        arcs += [(nodes[i], nodes[i + 1], caps[i]) for i in range(L + 1)]
        want += min(caps)
    g = W.from_arcs(V, arcs, s, t)
    for r in solve_both(g):
        assert r.value == want
        certify(g, r)


@pytest.mark.parametrize("a,b", [(1, 1), (3, 5), (8, 2), (20, 20), (40, 17)])
def test_complete_bipartite_unit(a, b):
    s, t = a + b, a + b + 1
    arcs = [(s, i, 1) for i in range(a)] + [(a + j, t, 1) for j in range(b)]
    arcs += [(i, a + j, 1) for i in range(a) for j in range(b)]
    g = W.from_arcs(a + b + 2, arcs, s, t)
    for r in solve_both(g):
        assert r.value == min(a, b)
        certify(g, r)


def test_grid_with_zero_nlinks():
    g = W.grid(16, 12, seed=9)
    g.cap[:] = np.where(g.col[:] < 16 * 12, 0, g.cap)  # zero every pixel-to-pixel arc
    src = W.arc_sources(g)
    cs = np.zeros(g.V, np.int64)
    ct = np.zeros(g.V, np.int64)
    m_s = src == g.s
    cs[g.col[m_s]] = g.cap[m_s]
    m_t = g.col == g.t
    ct[src[m_t]] = g.cap[m_t]
    want = int(np.minimum(cs, ct)[: 16 * 12].sum())
    for r in solve_both(g):
        assert r.value == want
        certify(g, r)


def test_star_and_degenerate_cases():
    # star s -> v_i -> t
    caps_in, caps_out = [4, 0, 9, 3], [2, 5, 9, 8]
    arcs = [(0, i + 2, c) for i, c in enumerate(caps_in)] + [(i + 2, 1, c) for i, c in enumerate(caps_out)]
    g = W.from_arcs(6, arcs, 0, 1)
    for r in solve_both(g):
        assert r.value == sum(min(x, y) for x, y in zip(caps_in, caps_out))
    # unreachable sink
    g = W.from_arcs(4, [(0, 1, 5), (1, 2, 5), (3, 1, 7)], 0, 3)
    for r in solve_both(g):
        assert r.value == 0
        c = certify(g, r)
        assert c.side.tolist() == [0, 0, 0, 1]
    # single arc and parallel arcs s -> t, a self-loop and a reverse arc t -> s
    g = W.from_arcs(2, [(0, 1, 7), (0, 1, 5), (0, 0, 9), (1, 0, 4)], 0, 1)
    for r in solve_both(g):
        assert r.value == 12
        certify(g, r)
    # no arcs at all
    g = W.from_arcs(3, [], 0, 2)
    for r in solve_both(g):
        assert r.value == 0


def test_large_capacities_int64_excess():
    # many max-int32 arcs out of s: total excess exceeds 2^31
    k = 6
    arcs = [(0, 2 + i, 2**31 - 1) for i in range(k)] + [(2 + i, 1, 2**31 - 1) for i in range(k)]
    g = W.from_arcs(k + 2, arcs, 0, 1)
    for r in solve_both(g):
        assert r.value == k * (2**31 - 1)
        certify(g, r)


def _scipy_value(g):
    src = W.arc_sources(g)
    keep = src != g.col
    m = sp.csr_matrix((g.cap[keep].astype(np.int32), (src[keep], g.col[keep])), shape=(g.V, g.V))
    m.sum_duplicates()
    return int(maximum_flow(m, g.s, g.t, method="dinic").flow_value)


@pytest.mark.parametrize("seed", range(10))
def test_against_scipy_maximum_flow(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(50, 800))
    g = W.multigraph(V, int(rng.integers(V, 8 * V)), cmax=int(rng.integers(1, 200)), seed=seed + 77)
    a, b = solve_both(g)
    want = _scipy_value(g)
    assert a.value == want and b.value == want
    certify(g, a)
    certify(g, b)


@pytest.mark.parametrize("L,R,narcs,seed", [(200, 150, 2000, 1), (2000, 2000, 30000, 2), (5000, 3000, 60000, 3)])
def test_bipartite_equals_hopcroft_karp(L, R, narcs, seed):
    g = W.bipartite(L, R, narcs, 2.1, seed)
    src = W.arc_sources(g)
    m = src < L
    adj = sp.csr_matrix((np.ones(int(m.sum()), np.int8), (src[m], g.col[m] - L)), shape=(L, R))
    adj.sum_duplicates()
    match = maximum_bipartite_matching(adj, perm_type="column")
    want = int((match >= 0).sum())
    a, b = solve_both(g)
    assert a.value == want and b.value == want
    certify(g, a)


def test_full_size_bipartite_workload():
    """The 50k+50k Zipf bipartite workload: value equals Hopcroft-Karp at full size."""
    g = W.config_bipartite()
    L = 50_000
    src = W.arc_sources(g)
    m = src < L
    adj = sp.csr_matrix((np.ones(int(m.sum()), np.int8), (src[m], g.col[m] - L)), shape=(L, 50_000))
    adj.sum_duplicates()
    want = int((maximum_bipartite_matching(adj, perm_type="column") >= 0).sum())
    a, b = solve_both(g)
    assert a.value == want == b.value
    certify(g, a)


def test_certificate_rejects_planted_mistakes():
    g = W.config_plain()
    r = oracle.dinic(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    ok = certify(g, r)
    # capacity violation
    i = int(np.argmax(r.flow == g.cap))
    bad = r.flow.copy()
    bad[i] += 1
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, bad)
    assert c.code == 1 and c.bad == i
    # negative flow
    bad = r.flow.copy()
    j = int(np.argmax(r.flow == 0))
    bad[j] = -1
    assert oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, bad).code == 1
    # conservation violation at an interior vertex
    src = W.arc_sources(g)
    k = int(np.argmax((r.flow > 0) & (src != g.s) & (g.col != g.t)))
    bad = r.flow.copy()
    bad[k] -= 1
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, bad)
    assert c.code == 2
    # feasible but not maximum: the zero flow
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, np.zeros_like(r.flow))
    assert c.feasible and c.value == 0 and not c.is_maximum(g.s)
    # a flow cycle added on top of a maximum flow keeps it maximum and keeps the side
    assert ok.value == r.value


def test_generators_are_deterministic():
    a = W.config_plain()
    b = W.config_plain()
    assert a.sha256() == b.sha256()
    assert W.random_graph(1000, 8000, 1, 100, 2).sha256() != a.sha256()
    g = W.rmat(12, seed=5)
    assert g.sha256() == W.rmat(12, seed=5).sha256()
    src = W.arc_sources(g)
    assert not np.any(src == g.col)  # self-loops removed
    key = src.astype(np.int64) * g.V + g.col
    assert np.unique(key).size == g.E  # duplicates removed
    assert g.cap.min() >= 1 and g.cap.max() <= 1000
