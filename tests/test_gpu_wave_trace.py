"""Per-wave trace: the paper's workload analysis (section 5) times every warp
from its first thread; here the first lane of every wave of every sweep
launch records its execution time and work.

Checks: tracing changes no result; the records account for exactly the arc
scans the solve counted; and the paper's observation on a bipartite graph
with hub vertices: the vertex-centric kernel spreads execution time over the
waves that have work more evenly (lower standard deviation of the times
normalised by their launch's mean) than the thread-centric kernel.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu

WATCHDOG = dict(max_wall_ms=120_000)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def spread(tr):
    """Std-dev of per-wave times normalised by the mean of their launch, over waves with work."""
    busy = tr[tr[:, 4] > 0]
    norm = []
    for key in np.unique(busy[:, 0] * 4 + busy[:, 1]):
        t = busy[busy[:, 0] * 4 + busy[:, 1] == key, 2].astype(np.float64)
        if len(t) > 1 and t.mean() > 0:
            norm.append(t / t.mean())
    return float(np.concatenate(norm).std())


def _solve_traced(g, **opts):
    from paper_2404_00270_amd import wbpr

    with wbpr.Solver(0, wave_trace=1, **opts, **WATCHDOG) as s:
        r = s.solve(g)
        tr = s.wave_trace()
    return r, tr


@pytest.mark.parametrize("lanes", [0, 1])
def test_trace_is_exact_and_harmless(lanes):
    g = W.random_graph(5000, 60000, 1, 100, 81)
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    r, tr = _solve_traced(g, lanes_per_vertex=lanes)
    say(f"[trace] lanes={lanes} records={len(tr)} sweeps={r.stats['sweeps']}")
    assert r.value == ref[0] and np.array_equal(r.side, ref[1])
    assert len(tr) > 0
    assert set(np.unique(tr[:, 1])) <= {0, 1, 2, 3}
    assert tr[:, 0].min() >= 0 and tr[:, 0].max() < r.stats["sweeps"]
    assert (tr[:, 2] >= 0).all() and (tr[:, 3] >= 0).all() and (tr[:, 4] >= 0).all()
    assert int(tr[:, 3].sum()) == r.stats["arc_scans"]
    if lanes == 1:  # thread-centric: short-row tiles only
        assert set(np.unique(tr[:, 1])) == {0}


def test_untraced_solve_reports_nothing():
    from paper_2404_00270_amd import wbpr

    g = W.config_plain()
    with wbpr.Solver(0, **WATCHDOG) as s:
        s.solve(g)
        assert len(s.wave_trace()) == 0


def test_vertex_centric_balances_waves_on_hubs():
    g = W.WORKLOADS["bipartite"]()
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)[0]
    rv, tv = _solve_traced(g)
    rt, tt = _solve_traced(g, lanes_per_vertex=1)
    assert rv.value == ref and rt.value == ref
    sv, st = spread(tv), spread(tt)
    say(f"[trace] bipartite spread: VC {sv:.3f} ({len(tv)} records), TC {st:.3f} ({len(tt)} records)")
    assert sv < st
