"""GPU tests of the multi-terminal front end (the paper's experimental
protocol, section 4: BFS-chosen source/sink pairs among the vertices farthest
apart, joined by a super-source and a super-sink).

The BFS eccentricities are compared with scipy's breadth-first distances,
the pair rule is replayed from its definition (SplitMix64 draws, 4k
candidates, decreasing eccentricity), and the multi-terminal flow is checked
against the oracle on a super-source/super-sink graph that the test builds
itself.
"""
import sys

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu

WATCHDOG = dict(max_wall_ms=120_000)
M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_2404_00270_amd import wbpr

    s = wbpr.Solver(0, **WATCHDOG)
    yield s
    s.close()


def bfs_reference(g, sources):
    """Eccentricity and smallest farthest vertex by scipy's unweighted BFS over arcs of positive capacity."""
    u = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    keep = (g.cap > 0) & (u != g.col)
    A = csr_matrix((np.ones(int(keep.sum())), (u[keep], g.col[keep])), shape=(g.V, g.V))
    d = shortest_path(A, method="D", directed=True, unweighted=True, indices=np.asarray(sources))
    ecc, far = [], []
    for i, s in enumerate(sources):
        row = d[i]
        fin = np.isfinite(row)
        e = int(row[fin].max())
        ecc.append(e)
        far.append(int(np.flatnonzero(fin & (row == e)).min()) if e > 0 else int(s))
    return np.array(ecc), np.array(far)


def splitmix64(x):
    """SplitMix64 (Steele, Lea and Flood 2014): (new state, output)."""
    x = (x + 0x9E3779B97F4A7C15) & M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return x, z ^ (z >> 31)


def pick_reference(g, k, seed):
    u = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    out_pos = np.zeros(g.V, bool)
    out_pos[u[(g.cap > 0) & (u != g.col)]] = True
    want = min(4 * k, int(out_pos.sum()))
    cand, drawn, x, tries = [], set(), seed, 0
    while len(cand) < want and tries < 64 * want:
        x, z = splitmix64(x)
        v = z % g.V
        tries += 1
        if out_pos[v] and v not in drawn:
            drawn.add(v)
            cand.append(int(v))
    if not cand:
        return [], []
    ecc, far = bfs_reference(g, cand)
    order = sorted(range(len(cand)), key=lambda i: -ecc[i])  # stable: draw order on ties
    used, src, snk = set(), [], []
    for i in order:
        if len(src) == k or ecc[i] == 0:
            break
        if cand[i] in used or far[i] in used:
            continue
        used |= {cand[i], int(far[i])}
        src.append(cand[i])
        snk.append(int(far[i]))
    return src, snk


def augmented(g, sources, sinks):
    """Super-source V and super-sink V + 1, built here independently of the library."""
    u = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    real = u != g.col
    out_cap = np.bincount(u[real], weights=g.cap[real], minlength=g.V).astype(np.int64)
    in_cap = np.bincount(g.col[real], weights=g.cap[real], minlength=g.V).astype(np.int64)
    arcs = list(zip(u.tolist(), g.col.tolist(), g.cap.tolist()))
    arcs += [(g.V, int(s), int(out_cap[s])) for s in sources]
    arcs += [(int(t), g.V + 1, int(in_cap[t])) for t in sinks]
    return W.from_arcs(g.V + 2, arcs, g.V, g.V + 1, g.name + "+ST"), len(g.col)


def check_multi(g, sources, sinks, r):
    ga, E = augmented(g, sources, sinks)
    value, side, _ = oracle.reference(ga.V, ga.row_ptr, ga.col, ga.cap, ga.s, ga.t)
    assert r.value == value, (g.name, r.value, value)
    assert np.array_equal(r.side, side[: g.V])
    # complete the flow with the super-arcs (net out of each source, into each sink)
    u = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    net = np.bincount(u, weights=r.flow, minlength=g.V) - np.bincount(g.col, weights=r.flow, minlength=g.V)
    ua = np.repeat(np.arange(ga.V), np.diff(ga.row_ptr))
    fa = np.zeros(len(ga.col), np.int64)
    # from_arcs keeps list order inside a row: the original arcs come first in every row
    pos = {}
    for i, (a, b) in enumerate(zip(ua.tolist(), ga.col.tolist())):
        pos.setdefault((a, b), []).append(i)
    for i, (a, b) in enumerate(zip(u.tolist(), g.col.tolist())):
        fa[pos[(a, b)].pop(0)] = r.flow[i]
    for s in sources:
        fa[pos[(g.V, int(s))].pop(0)] = net[s]
    for t in sinks:
        fa[pos[(int(t), g.V + 1)].pop(0)] = -net[t]
    c = oracle.check(ga.V, ga.row_ptr, ga.col, ga.cap, ga.s, ga.t, fa.astype(np.int32))
    assert c.feasible and c.value == value and c.cut_capacity == value, (c.code, c.bad)


@pytest.mark.parametrize("make", [
    lambda: W.random_graph(3000, 15000, 1, 100, 91),
    lambda: W.multigraph(400, 1600, cmax=5, seed=92),   # zero capacities and self-loops
    lambda: W.grid(40, 30, seed=93),
])
def test_bfs_farthest_matches_breadth_first_distances(solver, make):
    g = make()
    rng = np.random.default_rng(7)
    src = rng.choice(g.V, size=min(g.V, 150), replace=False).astype(np.int32)  # three passes of 64
    ecc, far = solver.bfs_farthest(g, src)
    say(f"[bfs] {g.name}: ecc max {ecc.max()}")
    re, rf = bfs_reference(g, src)
    assert np.array_equal(ecc, re)
    assert np.array_equal(far, rf)


def test_pick_terminals_follows_the_rule(solver):
    for g, k, seed in ((W.random_graph(2000, 8000, 1, 50, 94), 5, 11), (W.grid(30, 30, seed=95), 20, 12),
                       (W.multigraph(60, 100, cmax=3, seed=96), 8, 13)):
        src, snk = solver.pick_terminals(g, k, seed)
        rs, rt = pick_reference(g, k, seed)
        say(f"[pick] {g.name}: {len(src)} pairs")
        assert src.tolist() == rs and snk.tolist() == rt
        assert len(set(src.tolist()) | set(snk.tolist())) == 2 * len(src)


@pytest.mark.parametrize("make,k", [
    (lambda: W.random_graph(3000, 24000, 1, 100, 97), 6),
    (lambda: W.grid(48, 40, seed=98), 20),
    (lambda: W.bipartite(800, 600, 6000, 2.1, 99), 10),
])
def test_solve_multi_matches_oracle(solver, make, k):
    g = make()
    src, snk = solver.pick_terminals(g, k, 5)
    assert len(src) > 0
    say(f"[multi] {g.name}: {len(src)} pairs")
    check_multi(g, src, snk, solver.solve_multi(g, src, snk))


def test_solve_multi_closed_form(solver):
    # k disjoint two-arc paths s_i -> a_i -> t_i: the flow is the sum of the path minima
    rng = np.random.default_rng(3)
    k = 7
    caps = rng.integers(1, 1000, size=(k, 2))
    arcs = [(3 * i, 3 * i + 1, int(caps[i, 0])) for i in range(k)] + [(3 * i + 1, 3 * i + 2, int(caps[i, 1]))
                                                                       for i in range(k)]
    g = W.from_arcs(3 * k, arcs, 0, 2, "paths")
    r = solver.solve_multi(g, [3 * i for i in range(k)], [3 * i + 2 for i in range(k)])
    assert r.value == int(caps.min(axis=1).sum())


def test_solve_multi_errors(solver):
    from paper_2404_00270_amd import wbpr

    g = W.random_graph(100, 500, 1, 10, 5)
    assert solver.solve_multi(g, [1, 2], [3, 4]).value >= 0
    rc = wbpr.wbpr_solve_multi(solver.ctx, g, [1, 2], [2, 4], return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    rc = wbpr.wbpr_solve_multi(solver.ctx, g, [1, 1], [3, 4], return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    rc = wbpr.wbpr_solve_multi(solver.ctx, g, [1], [100], return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    big = W.from_arcs(4, [(0, 1, 2**31 - 1), (0, 2, 2**31 - 1), (1, 3, 5), (2, 3, 5)], 0, 3)
    rc = wbpr.wbpr_solve_multi(solver.ctx, big, [0], [3], return_code=True)
    assert rc == wbpr.WBPR_EOVERFLOW
    # still usable
    check_multi(g, [1, 2], [3, 4], solver.solve_multi(g, [1, 2], [3, 4]))
