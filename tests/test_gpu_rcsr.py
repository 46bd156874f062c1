"""GPU parity of the RCSR layout (paper, section 3.2: forward CSR plus a
reversed CSR whose entries index the arc's flow).

The same bar as the BCSR tests: every result equals the oracle's (value and
canonical sink side, bit for bit) and every per-arc flow passes the oracle's
certificate, over multigraphs with parallel and antiparallel arcs, self-loops
and zero capacities, every tile width and tier split, the thread-centric
kernel, the full-scan queue, the paper's single-push mode, fixed relabel
frequencies, batches, the server, uploaded graphs (residual reset) and the
full-size workloads.  RCSR never merges arcs, so parallel capacities that sum
past INT32_MAX solve instead of being rejected.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "workload_values.json")
RCSR = 2
OPTS = dict(layout=RCSR, max_wall_ms=120_000)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_2404_00270_amd import wbpr

    s = wbpr.Solver(0, **OPTS)
    yield s
    s.close()


def check_against_oracle(g, res, ref=None):
    if ref is None:
        ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    value, side, cutcap = ref
    assert res.value == value, (g.name, res.value, value)
    if res.side is not None:
        assert np.array_equal(res.side, side), (g.name, int(res.side.sum()), int(side.sum()))
    if res.flow is not None:
        c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, res.flow)
        assert c.feasible, (g.name, c.code, c.bad)
        assert c.value == value and c.cut_capacity == value
        assert np.array_equal(c.side, side)


@pytest.mark.parametrize("seed", range(40))
def test_small_multigraphs_rcsr(solver, seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 40))
    E = int(rng.integers(0, 6 * V))
    g = W.multigraph(V, E, cmax=int(rng.integers(0, 30)), seed=5000 + seed)
    say(f"[rcsr-small] seed={seed} V={V} E={E}")
    r = solver.solve(g)
    assert r.stats["lds_solved"] == 0  # RCSR instances take the rounds
    check_against_oracle(g, r)


@pytest.mark.parametrize("V,E,seed", [(100, 600, 1), (1000, 8000, 2), (3000, 40000, 3), (20000, 100000, 4)])
def test_random_graphs_ragged_rcsr(solver, V, E, seed):
    g = W.random_graph(V, E, 1, 100, seed)
    say(f"[rcsr-random] V={V} E={E}")
    r = solver.solve(g)
    assert r.stats["M"] == 2 * E  # one forward and one reverse entry per arc
    check_against_oracle(g, r)


def test_degenerate_cases_rcsr(solver):
    cases = [
        W.from_arcs(2, [], 0, 1, "no-arcs"),
        W.from_arcs(2, [(0, 1, 7)], 0, 1, "single-arc"),
        W.from_arcs(2, [(0, 1, 7), (0, 1, 5), (0, 0, 9), (1, 0, 4), (1, 1, 3)], 0, 1, "parallel+loops"),
        W.from_arcs(4, [(0, 1, 5), (1, 2, 5), (3, 1, 7)], 0, 3, "sink-unreachable"),
        W.from_arcs(4, [(1, 2, 5), (2, 3, 5)], 0, 3, "source-isolated"),
        W.from_arcs(5, [(0, 1, 0), (1, 4, 3), (0, 2, 3), (2, 4, 0)], 0, 4, "zero-caps"),
        W.from_arcs(3, [(0, 1, 3), (1, 0, 3), (1, 2, 2), (2, 1, 9)], 2, 0, "reverse-roles"),
        W.from_arcs(8, [(0, 2 + i, 2**31 - 1) for i in range(6)] + [(2 + i, 1, 2**31 - 1) for i in range(6)], 0, 1,
                    "int64-excess"),
        # parallel capacities past INT32_MAX (BCSR rejects the merged entry; RCSR keeps the arcs apart)
        W.from_arcs(3, [(0, 1, 2**22)] * 600 + [(1, 2, 2**22)] * 600, 0, 2, "parallel-past-int32"),
        W.from_arcs(3, [(0, 1, 2**31 - 1), (1, 0, 5), (1, 2, 4)], 0, 2, "antiparallel-int32-max"),
    ]
    for g in cases:
        say(f"[rcsr-degenerate] {g.name}")
        check_against_oracle(g, solver.solve(g))


def test_long_path_and_star_rcsr(solver):
    n = 3000
    g = W.from_arcs(n, [(i, i + 1, 1 + (i * 7919) % 50) for i in range(n - 1)], 0, n - 1, "path")
    check_against_oracle(g, solver.solve(g))
    k = 5000
    arcs = [(0, 2 + i, 1 + i % 9) for i in range(k)] + [(2 + i, 1, 1 + (i * 31) % 7) for i in range(k)]
    g = W.from_arcs(k + 2, arcs, 0, 1, "star")
    check_against_oracle(g, solver.solve(g))


@pytest.mark.parametrize("lanes", [1, 4, 8, 16, 32, 64])
def test_every_tile_width_and_split_path_rcsr(solver, lanes):
    g = W.bipartite(3000, 2000, 40000, 2.1, 11)
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    for mode in (1, 2):
        for split, block in ((0, 0), (1, 2), (7, 60)):
            say(f"[rcsr-tiles] lanes={lanes} split={split} block={block} push_mode={mode}")
            solver.set_options(lanes_per_vertex=lanes, split_degree=split, block_degree=block, push_mode=mode,
                               **OPTS)
            try:
                check_against_oracle(g, solver.solve(g), ref)
            finally:
                solver.set_options(**OPTS)


@pytest.mark.parametrize("lanes,avq_mode,push_mode", [(1, 1, 1), (1, 0, 2), (0, 1, 2), (8, 1, 1)])
def test_thread_centric_and_full_scan_queue_rcsr(solver, lanes, avq_mode, push_mode):
    graphs = [W.bipartite(3000, 2000, 40000, 2.1, 11), W.random_graph(2000, 16000, 1, 100, 21)]
    graphs += [W.multigraph(int(v), int(6 * v), cmax=25, seed=300 + int(v)) for v in (2, 7, 33, 120)]
    solver.set_options(lanes_per_vertex=lanes, avq_mode=avq_mode, push_mode=push_mode, **OPTS)
    try:
        for g in graphs:
            say(f"[rcsr-tc/scan] lanes={lanes} avq={avq_mode} push={push_mode} {g.name}")
            check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**OPTS)


@pytest.mark.parametrize("seed", range(12))
def test_paper_single_push_mode_rcsr(solver, seed):
    rng = np.random.default_rng(100 + seed)
    V = int(rng.integers(2, 60))
    g = W.multigraph(V, int(rng.integers(0, 8 * V)), cmax=int(rng.integers(0, 40)), seed=7000 + seed)
    solver.set_options(push_mode=1, **OPTS)
    try:
        check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**OPTS)


@pytest.mark.parametrize("K", [1, 3, 64])
def test_global_relabel_frequency_rcsr(solver, K):
    g = W.random_graph(2000, 16000, 1, 100, 21)
    solver.set_options(gr_every_sweeps=K, **OPTS)
    try:
        check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**OPTS)


def test_error_paths_rcsr(solver):
    from paper_2404_00270_amd import wbpr

    g = W.config_plain()
    ctx = solver.ctx
    bad = g.col.copy()
    bad[17] = g.V + 3
    assert wbpr.wbpr_solve(ctx, g.V, g.row_ptr, bad, g.cap, g.s, g.t, return_code=True) == wbpr.WBPR_EINVAL
    neg = g.cap.copy()
    neg[5] = -1
    assert wbpr.wbpr_solve(ctx, g.V, g.row_ptr, g.col, neg, g.s, g.t, return_code=True) == wbpr.WBPR_EINVAL
    rp = g.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]
    if rp[10] != rp[11]:
        assert wbpr.wbpr_solve(ctx, g.V, rp, g.col, g.cap, g.s, g.t, return_code=True) == wbpr.WBPR_EINVAL
    rp = g.row_ptr.copy()
    rp[20] = g.E + 5000  # beyond E: rejected, nothing written out of range
    assert wbpr.wbpr_solve(ctx, g.V, rp, g.col, g.cap, g.s, g.t, return_code=True) == wbpr.WBPR_EINVAL
    check_against_oracle(g, solver.solve(g))  # the context still works


def test_batch_server_and_uploaded_rcsr():
    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(3)
    gs = [W.multigraph(int(rng.integers(2, 50)), int(rng.integers(0, 200)), cmax=25, seed=800 + i) for i in range(8)]
    gs += [W.batch_instance(40 + i, vmin=64, vmax=8192) for i in range(8)]
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    with wbpr.Solver(0, **OPTS) as s:
        say(f"[rcsr-batch] n={len(gs)}")
        res = s.solve_batch(gs)
        for i, g in enumerate(gs):
            assert res.values[i] == refs[i][0], (i, g.name)
            assert np.array_equal(res.sides[i], refs[i][1])
            c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, res.flows[i])
            assert c.feasible and c.value == refs[i][0]
        say("[rcsr-server]")
        with wbpr.Server(s, hbm_budget_bytes=48 << 20, want_flows=True, want_sides=True) as srv:
            tickets = [srv.submit(g) for g in gs]
            for i, (g, tk) in enumerate(zip(gs, tickets)):
                r = srv.wait(tk, 60_000)
                assert r is not None and r.status == 0
                assert r.value == refs[i][0] and np.array_equal(r.side, refs[i][1])
                c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
                assert c.feasible and c.value == refs[i][0]
        say("[rcsr-uploaded]")
        g0 = W.random_graph(3000, 24000, 1, 100, 9)
        with wbpr.UploadedGraph(s, g0) as ug:
            for (src, snk) in ((0, 2999), (5, 17), (2999, 0), (100, 2000)):
                g = W.Graph(g0.V, g0.row_ptr, g0.col, g0.cap, src, snk, f"pair-{src}-{snk}")
                check_against_oracle(g, ug.solve(src, snk))


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["plain", "bipartite", "grid", "rmat"])
def test_full_size_workloads_rcsr(solver, name):
    gold = _golden()[name]
    g = W.WORKLOADS[name]()
    assert g.sha256() == gold["graph_sha256"]
    say(f"[rcsr-full] solving {name} V={g.V} E={g.E}")
    r = solver.solve(g)
    say(f"[rcsr-full] {name} value={r.value} sweeps={r.stats['sweeps']} relabels={r.stats['global_relabels']} "
        f"ms={r.stats['ms_total']:.1f}")
    assert r.value == gold["value"]
    assert int(r.side.sum()) == gold["sink_side_size"]
    assert hashlib.sha256(r.side.tobytes()).hexdigest() == gold["sink_side_sha256"]
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
    assert c.feasible and c.value == gold["value"] and c.cut_capacity == gold["cut_capacity"]
