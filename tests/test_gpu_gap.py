"""GPU parity with the gap heuristic (option `gap`, on unless negative).

The heuristic is not part of the paper's method: between global relabels it
keeps a count of vertices per height and, once a height empties, leaves the
vertices above it to the next global relabel.  Results must stay exactly the
oracle's (flow value, canonical sink side, certified per-arc flow).
"""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2404_00270_amd import workloads as W

from test_gpu_parity import WATCHDOG, _golden, check_against_oracle, say

pytestmark = pytest.mark.gpu


def _bottleneck(nc=200, seed=3):
    """s feeds a dense cluster that reaches t only through one unit arc a -> t:
    once a -> t is saturated, a relabels and the height just above t empties."""
    rng = np.random.default_rng(seed)
    s, t, a, c0 = 0, 1, 2, 3
    arcs = [(s, c0 + i, 1000) for i in range(nc)]
    arcs += [(c0 + int(x), c0 + int(y), 1000) for x, y in rng.integers(0, nc, (10 * nc, 2)) if x != y]
    arcs += [(c0 + i, a, 1000) for i in range(0, nc, 4)]
    arcs += [(a, t, 1)]
    return W.from_arcs(c0 + nc, arcs, s, t, "bottleneck")


def test_gap_fires_on_a_bottleneck():
    from paper_2404_00270_amd import wbpr

    g = _bottleneck()
    with wbpr.Solver(0, lds_max_v=-1, gap=1, **WATCHDOG) as s:
        r = s.solve(g)
    say(f"[gap] bottleneck value={r.value} skipped={r.stats['gap_skipped']} sweeps={r.stats['sweeps']}")
    assert r.value == 1
    assert r.stats["gap_skipped"] > 0
    check_against_oracle(g, r)
    with wbpr.Solver(0, lds_max_v=-1, gap=-1, **WATCHDOG) as s:
        r0 = s.solve(g)
    assert r0.stats["gap_skipped"] == 0
    check_against_oracle(g, r0)


def _families():
    gs = [W.random_graph(2000, 16000, 1, 100, 21), W.random_graph(20000, 100000, 1, 100, 4),
          W.bipartite(3000, 2000, 40000, 2.1, 11), W.grid(64, 64, seed=5), W.grid(150, 97, seed=6),
          W.rmat(12, 16, seed=7), _bottleneck(400, 8)]
    gs += [W.multigraph(int(v), int(6 * v), cmax=25, seed=400 + int(v)) for v in (2, 7, 33, 120, 900)]
    return gs


@pytest.mark.parametrize("push_mode,avq_mode", [(0, 0), (1, 0), (0, 1)])
def test_gap_parity_families(push_mode, avq_mode):
    from paper_2404_00270_amd import wbpr

    with wbpr.Solver(0, lds_max_v=-1, gap=1, push_mode=push_mode, avq_mode=avq_mode, **WATCHDOG) as s:
        for g in _families():
            say(f"[gap] push={push_mode} avq={avq_mode} {g.name} V={g.V} E={g.E}")
            check_against_oracle(g, s.solve(g))


@pytest.mark.parametrize("seed", range(0, 40, 3))
def test_gap_small_multigraphs(seed):
    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 60))
    g = W.multigraph(V, int(rng.integers(0, 8 * V)), cmax=int(rng.integers(0, 40)), seed=9000 + seed)
    say(f"[gap-small] seed={seed} V={V}")
    with wbpr.Solver(0, lds_max_v=-1, gap=1, **WATCHDOG) as s:
        check_against_oracle(g, s.solve(g))


@pytest.mark.parametrize("name", ["bipartite", "grid", "rmat"])
def test_gap_full_size_workloads(name):
    from paper_2404_00270_amd import wbpr
    import oracle

    gold = _golden()[name]
    g = W.WORKLOADS[name]()
    with wbpr.Solver(0, gap=1, **WATCHDOG) as s:
        r = s.solve(g)
    say(f"[gap-full] {name} value={r.value} skipped={r.stats['gap_skipped']} "
        f"sweeps={r.stats['sweeps']} relabels={r.stats['global_relabels']} ms={r.stats['ms_total']:.1f}")
    assert r.value == gold["value"]
    assert int(r.side.sum()) == gold["sink_side_size"]
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
    assert c.feasible and c.value == gold["value"] and c.cut_capacity == gold["cut_capacity"]
    assert np.array_equal(c.side, r.side)


def test_gap_in_batches():
    """Per-height counts need one root: in a batch the heuristic runs only
    while a single instance is still in its phase (the others finished), and
    every instance gets exactly the oracle's result."""
    from paper_2404_00270_amd import wbpr

    gs = [W.random_graph(3000, 24000, 1, 100, 31 + i) for i in range(3)] + [_bottleneck(300, 9)]
    with wbpr.Solver(0, lds_max_v=-1, gap=1, **WATCHDOG) as s:
        br = s.solve_batch(gs)
    say(f"[gap-batch] skipped={br.stats['gap_skipped']}")
    for i, g in enumerate(gs):
        check_against_oracle(g, SimpleNamespace(value=int(br.values[i]), flow=br.flows[i], side=br.sides[i]))
