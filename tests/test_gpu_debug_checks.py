"""Option debug_checks: before every global relabel the preflow invariants of
section 2.2 are checked on the device (residuals not negative, each pair of
entries keeping its capacity, every vertex other than s and t holding exactly
its inflow minus its outflow).

* Clean solves pass every check in both layouts, in single solves, batches
  and the server, and their results still equal the oracle's.
* A violation planted from the host (one unit of excess added to a vertex
  before the first check, WBPR_DEBUG_PLANT) is reported: the solve fails with
  WBPR_EINTERNAL and a message naming one vertex.
"""
import subprocess
import sys
import os

import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)


def check(g, r):
    value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    assert r.value == value, (g.name, r.value, value)
    assert np.array_equal(r.side, side)
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
    assert c.feasible and c.value == value and c.cut_capacity == value


@pytest.mark.parametrize("layout", [1, 2])
def test_clean_solves_pass_every_check(layout):
    from paper_2404_00270_amd import wbpr

    with wbpr.Solver(0, layout=layout, debug_checks=1, max_wall_ms=60_000) as solver:
        for seed in range(6):
            rng = np.random.default_rng(seed)
            V = int(rng.integers(3, 60))
            g = W.multigraph(V, int(rng.integers(V, 6 * V)), cmax=25, seed=900 + seed)
            say(f"[debug] layout={layout} multigraph seed={seed} V={g.V} E={g.E}")
            r = solver.solve(g)
            assert r.stats["debug_checked"] == r.stats["global_relabels"] >= 1
            assert r.stats["lds_solved"] == 0 and r.stats["wg_solved"] == 0
            check(g, r)
        for V, E, seed in [(2000, 16000, 1), (30000, 200000, 2)]:
            g = W.random_graph(V, E, 1, 100, seed)
            say(f"[debug] layout={layout} random V={V} E={E}")
            r = solver.solve(g)
            assert r.stats["debug_checked"] == r.stats["global_relabels"] >= 1
            check(g, r)
        g = W.bipartite(3000, 3000, 40000, seed=7)
        say(f"[debug] layout={layout} bipartite V={g.V}")
        r = solver.solve(g)
        assert r.stats["debug_checked"] >= 1
        check(g, r)
        gs = [W.batch_instance(i, vmax=4096) for i in range(80)]
        say(f"[debug] layout={layout} batch of {len(gs)}")
        b = solver.solve_batch(gs)
        assert b.stats["debug_checked"] >= 1 and b.stats["wg_solved"] == 0
        for k, g in enumerate(gs):
            value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
            assert b.values[k] == value, k
            assert np.array_equal(b.sides[k], side), k


def test_server_with_checks():
    from paper_2404_00270_amd import wbpr

    gs = [W.batch_instance(i, vmax=2048) for i in range(24)]
    with wbpr.Solver(0, debug_checks=1, max_wall_ms=60_000) as solver:
        with wbpr.Server(solver, want_flows=True, want_sides=True) as srv:
            tickets = [srv.submit(g) for g in gs]
            for g, tk in zip(gs, tickets):
                r = srv.wait(tk, 60_000)
                assert r is not None and r.status == 0
                value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
                assert r.value == value and np.array_equal(r.side, side)


_PLANTED = r"""
import sys
sys.path.insert(0, {root!r})
from paper_2404_00270_amd import wbpr
from paper_2404_00270_amd import workloads as W
g = W.random_graph(500, 4000, 1, 100, 3)
with wbpr.Solver(0, layout={layout}, debug_checks=1, max_wall_ms=30_000) as s:
    try:
        s.solve(g)
    except wbpr.WbprError as e:
        print("ERR", e.code, str(e))
        sys.exit(0)
print("NOERR")
"""


@pytest.mark.parametrize("layout", [1, 2])
def test_planted_violation_is_reported(layout):
    env = dict(os.environ, WBPR_DEBUG_PLANT="1")
    say(f"[debug] planted violation, layout={layout}")
    out = subprocess.run([sys.executable, "-c", _PLANTED.format(root=ROOT, layout=layout)], env=env,
                         capture_output=True, text=True, timeout=120)
    say(out.stdout.strip(), out.stderr.strip()[-400:])
    assert out.returncode == 0
    line = [ln for ln in out.stdout.splitlines() if ln.startswith(("ERR", "NOERR"))][-1]
    assert line.startswith("ERR"), line
    from paper_2404_00270_amd import wbpr

    assert f"ERR {wbpr.WBPR_EINTERNAL}" in line
    assert "0 entries and 1 vertices violate" in line
