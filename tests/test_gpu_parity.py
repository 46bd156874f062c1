"""GPU parity: the HIP solver (through the C ABI) against the CPU oracle.

Exact comparisons: flow value (int64) and the canonical sink-side vector
(vertices that reach t in the residual graph) must equal the oracle's bit for
bit; the returned per-arc flow is not unique, so it must pass the oracle's
certificate (capacity bounds, conservation, value == capacity of the
returned cut).  Full-size workloads compare against tests/golden values
written by tests/golden/make_golden.py (oracle only).
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
WATCHDOG = dict(max_wall_ms=120_000)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def solver():
    from paper_2404_00270_amd import wbpr

    s = wbpr.Solver(0, **WATCHDOG)
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
        assert c.value == value
        assert c.cut_capacity == value
        assert np.array_equal(c.side, side)


def test_device_arch():
    from paper_2404_00270_amd import wbpr

    assert wbpr.wbpr_device_arch(0).startswith("gfx950")


@pytest.mark.parametrize("seed", range(60))
def test_small_multigraphs(solver, seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 40))
    E = int(rng.integers(0, 6 * V))
    g = W.multigraph(V, E, cmax=int(rng.integers(0, 30)), seed=5000 + seed)
    say(f"[small] seed={seed} V={V} E={E}")
    check_against_oracle(g, solver.solve(g))


@pytest.mark.parametrize("V,E,seed", [(100, 600, 1), (1000, 8000, 2), (3000, 40000, 3), (20000, 100000, 4)])
def test_random_graphs_ragged(solver, V, E, seed):
    g = W.random_graph(V, E, 1, 100, seed)
    say(f"[random] V={V} E={E} seed={seed}")
    check_against_oracle(g, solver.solve(g))


@pytest.mark.parametrize("V,E,seed", [(50_000, 3_000, 11), (300_000, 40_000, 12)])
def test_sparse_rows_spanning_many_empty_rows(solver, V, E, seed):
    """Most rows empty: the builder's tiles of 2,048 arcs span more rows than
    it keeps in LDS (2,048 row starts), so arcs find their rows by a search
    over the whole row_ptr, and empty rows sit at both ends."""
    rng = np.random.default_rng(seed)
    hi = V - V // 10
    u = rng.integers(V // 10, hi, E)
    v = rng.integers(V // 10, hi, E)
    arcs = [(int(a), int(b), int(c)) for a, b, c in zip(u, v, rng.integers(1, 100, E))]
    s, t = int(u[0]), int(v[-1])
    arcs += [(s, int(x), 1000) for x in u[1:50]] + [(int(x), t, 1000) for x in v[1:50]]
    g = _reorder_rows(W.from_arcs(V, arcs, s, t, f"sparse-{V}-{E}"))
    say(f"[sparse] V={V} E={g.E}")
    check_against_oracle(g, solver.solve(g))


def _reorder_rows(g, seed=None):
    """Same graph with each row's arcs sorted by column (seed None) or shuffled."""
    row = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    minor = g.col if seed is None else np.random.default_rng(seed).random(g.E)
    order = np.lexsort((minor, row))
    tag = "-sorted" if seed is None else "-shuffled"
    return W.Graph(g.V, g.row_ptr, g.col[order].copy(), g.cap[order].copy(), g.s, g.t, g.name + tag)


# both builder paths (column-sorted rows: backward-key sort + merge; any
# order: full sort), at 1, 2 and 3 radix passes over the row bits
@pytest.mark.parametrize("V,E,seed", [(200, 1500, 5), (5000, 40000, 6), (70000, 300000, 7)])
def test_sorted_and_unsorted_rows(solver, V, E, seed):
    g0 = W.multigraph(V, E, cmax=25, seed=seed)
    ref = oracle.reference(g0.V, g0.row_ptr, g0.col, g0.cap, g0.s, g0.t)
    for g in (_reorder_rows(g0), _reorder_rows(g0, seed)):
        say(f"[row-order] {g.name}")
        check_against_oracle(g, solver.solve(g), ref)


@pytest.mark.parametrize("E", [1, 2047, 2048, 2049, 6143, 6144, 6145, 12289])
def test_arc_counts_at_tile_boundaries(solver, E):
    """Arc counts around the key emission's tiles (2,048 arcs) and the radix
    sort's tiles (6,144 keys, three emission tiles): the emission counts the
    first radix pass's histogram per radix tile, so a last tile that is
    partial, or holds one emission tile only, must still give the sort's
    offsets.  Column-sorted rows (the path that uses that histogram) and
    shuffled rows (the full sort, which counts its own)."""
    g0 = W.random_graph(max(8, E // 6), E, 1, 100, 7)
    assert g0.E == E
    ref = oracle.reference(g0.V, g0.row_ptr, g0.col, g0.cap, g0.s, g0.t)
    for g in (_reorder_rows(g0), _reorder_rows(g0, 3)):
        say(f"[tiles] {g.name} E={E}")
        check_against_oracle(g, solver.solve(g), ref)


@pytest.mark.parametrize("seed", [1, 2])
def test_long_groups_of_parallel_arcs(solver, seed):
    """Pairs joined by hundreds of parallel and antiparallel arcs (groups of
    equal keys longer than one thread walks, up to several workgroup tiles)."""
    rng = np.random.default_rng(seed)
    V = 40
    arcs = []
    for (u, v), n in (((1, 2), 300), ((2, 1), 257), ((3, 4), 700), ((5, 6), 1500), ((6, 5), 40)):
        arcs += [(u, v, int(c)) for c in rng.integers(0, 1000, n)]
    for _ in range(400):
        u, v = (int(x) for x in rng.integers(0, V, 2))
        arcs.append((u, v, int(rng.integers(1, 5000))))
    # route s -> the long pairs -> t so that their capacities matter
    arcs += [(0, 1, 10**6), (0, 3, 10**6), (0, 5, 10**6), (2, V - 1, 10**6), (4, V - 1, 10**6), (6, V - 1, 10**6)]
    order = rng.permutation(len(arcs))
    g = W.from_arcs(V, [arcs[k] for k in order], 0, V - 1, f"long-groups-{seed}")
    say(f"[long-groups] seed={seed} E={g.E}")
    check_against_oracle(g, solver.solve(g))


def _longest_column_run(g):
    """Longest run of one column inside a row (rows sorted by column)."""
    row = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    same = (row[1:] == row[:-1]) & (g.col[1:] == g.col[:-1])
    best = run = 1 if g.E else 0
    for x in same:
        run = run + 1 if x else 1
        best = max(best, run)
    return best


@pytest.mark.parametrize("run", [256, 257])
def test_sorted_rows_with_runs_of_parallel_arcs(solver, run):
    """Column-sorted rows repeating columns up to `run` times, in both
    directions and as self-loops, among ~60k short groups (about 70 merge
    tiles of 2,048 keys): with runs of at most 256 the builder merges and
    finishes the entries in one kernel, moving each tile bound past a group
    of up to 512 equal keys; one run of 257 sends it through the general
    sorted path.  Both against the oracle."""
    rng = np.random.default_rng(run)
    V = 2000
    arcs, pairs = [], set()
    for k in range(24):
        while True:
            u, v = (int(x) for x in rng.integers(1, 200, 2))
            if u != v and (u, v) not in pairs and (v, u) not in pairs:
                break
        pairs.add((u, v))
        n1 = run if k % 4 == 0 else int(rng.integers(1, run + 1))
        n2 = run if k % 8 == 0 else int(rng.integers(0, run + 1))
        arcs += [(u, v, int(c)) for c in rng.integers(0, 1000, n1)]
        arcs += [(v, u, int(c)) for c in rng.integers(0, 1000, n2)]
    loops = set()
    for k in range(6):
        u = int(rng.integers(200, 300))
        if u not in loops:
            loops.add(u)
            arcs += [(u, u, int(c)) for c in rng.integers(0, 50, run if k == 0 else int(rng.integers(1, run + 1)))]
    taken = pairs | {(v, u) for u, v in pairs}
    for _ in range(60000):
        u, v = (int(x) for x in rng.integers(0, V, 2))
        if (u, v) in taken or (u == v and u in loops):
            continue
        arcs.append((u, v, int(rng.integers(1, 5000))))
    # s feeds the long pairs' tails and their heads drain to t
    for u, v in sorted(pairs):
        arcs += [(0, u, 10**6), (v, V - 1, 10**6), (0, v, 10**5), (u, V - 1, 10**5)]
    g = _reorder_rows(W.from_arcs(V, arcs, 0, V - 1, f"runs-{run}"))
    assert _longest_column_run(g) == run
    say(f"[runs] run={run} E={g.E}")
    check_against_oracle(g, solver.solve(g))


def test_long_group_overflow(solver):
    from paper_2404_00270_amd import wbpr

    # 600 parallel arcs of 2^22 sum past INT32_MAX; 500 of them do not
    for n, code in ((600, wbpr.WBPR_EOVERFLOW), (500, wbpr.WBPR_OK)):
        g = W.from_arcs(3, [(0, 1, 2**22)] * n + [(1, 2, 7)], 0, 2)
        rc = wbpr.wbpr_solve(solver.ctx, g.V, g.row_ptr, g.col, g.cap, 0, 2, return_code=True)
        assert rc == code, (n, rc)


@pytest.mark.parametrize("seed", range(0, 60, 4))
def test_small_multigraphs_through_rounds(seed):
    """The same small instances with the LDS-resident path off (rounds of launches)."""
    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 40))
    E = int(rng.integers(0, 6 * V))
    g = W.multigraph(V, E, cmax=int(rng.integers(0, 30)), seed=5000 + seed)
    with wbpr.Solver(0, lds_max_v=-1, **WATCHDOG) as s:
        r = s.solve(g)
    assert r.stats["lds_solved"] == 0
    check_against_oracle(g, r)


def test_lds_resident_path(solver):
    """Instances up to 1024 vertices that fit one workgroup's LDS are solved
    whole by it; larger ones, or lds_max_v = -1, take the rounds."""
    from paper_2404_00270_amd import wbpr

    # the first fits even a 64 KiB budget; the others need the 160 KiB of a CU
    for i, g in enumerate((W.random_graph(300, 2000, 1, 100, 76), W.random_graph(900, 7000, 1, 100, 77),
                           W.config_plain(), W.grid(30, 30, seed=8), W.bipartite(300, 300, 3000, 2.1, 9))):
        ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
        r = solver.solve(g)
        say(f"[lds] {g.name}: V={g.V} M={r.stats['M']} lds_solved={r.stats['lds_solved']} sweeps={r.stats['sweeps']}")
        if i == 0:
            assert r.stats["lds_solved"] == 1
        check_against_oracle(g, r, ref)
        v = solver.solve(g, want_flow=False)  # one phase only
        assert v.value == ref[0] and np.array_equal(v.side, ref[1])
    big = W.random_graph(5000, 40000, 1, 100, 78)
    assert solver.solve(big).stats["lds_solved"] == 0
    with wbpr.Solver(0, lds_max_v=100, **WATCHDOG) as s:
        g = W.random_graph(500, 4000, 1, 100, 79)
        r = s.solve(g)
        assert r.stats["lds_solved"] == 0
        check_against_oracle(g, r)


def test_lds_round_cap_hands_over_to_rounds(monkeypatch):
    """An LDS-resident solve that reaches its round cap writes nothing back
    and the rounds of launches finish the instance: forced from the host by
    a round cap of 1 (results must still equal the oracle's)."""
    from paper_2404_00270_amd import wbpr

    monkeypatch.setenv("WBPR_LDS_ROUND_CAP", "1")
    fallbacks = 0
    with wbpr.Solver(0, **WATCHDOG) as s:
        for seed in range(6):
            g = W.random_graph(200 + 100 * seed, 8 * (200 + 100 * seed), 1, 100, 300 + seed)
            r = s.solve(g)
            say(f"[lds-cap] {g.name}: lds_solved={r.stats['lds_solved']} fallbacks={r.stats['lds_fallbacks']}")
            assert r.stats["lds_solved"] + r.stats["lds_fallbacks"] == 1
            fallbacks += r.stats["lds_fallbacks"]
            check_against_oracle(g, r)
    assert fallbacks > 0


def test_degenerate_cases(solver):
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
    ]
    for g in cases:
        say(f"[degenerate] {g.name}")
        check_against_oracle(g, solver.solve(g))


def test_long_path_and_star(solver):
    n = 3000
    g = W.from_arcs(n, [(i, i + 1, 1 + (i * 7919) % 50) for i in range(n - 1)], 0, n - 1, "path")
    say("[path]")
    check_against_oracle(g, solver.solve(g))
    k = 5000  # hub rows far longer than the split threshold
    arcs = [(0, 2 + i, 1 + i % 9) for i in range(k)] + [(2 + i, 1, 1 + (i * 31) % 7) for i in range(k)]
    g = W.from_arcs(k + 2, arcs, 0, 1, "star")
    say("[star]")
    check_against_oracle(g, solver.solve(g))


@pytest.mark.parametrize("lanes", [4, 8, 16, 32, 64])
def test_every_tile_width_and_split_path(solver, lanes):
    g = W.bipartite(3000, 2000, 40000, 2.1, 11)
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    for mode in (1, 2):
        for split, block in ((0, 0), (1, 2), (7, 60), (3, 3)):
            say(f"[tiles] lanes={lanes} split={split} block={block} push_mode={mode}")
            solver.set_options(lanes_per_vertex=lanes, split_degree=split, block_degree=block, push_mode=mode,
                               **WATCHDOG)
            try:
                check_against_oracle(g, solver.solve(g), ref)
            finally:
                solver.set_options(**WATCHDOG)


@pytest.mark.parametrize("lanes,avq_mode,push_mode", [
    (1, 0, 2), (1, 0, 1), (1, 1, 2), (1, 1, 1),   # thread-centric, incremental / full-scan queue
    (0, 1, 2), (0, 1, 1), (8, 1, 2), (64, 1, 1),  # vertex-centric with the full-scan queue
])
def test_thread_centric_and_full_scan_queue(solver, lanes, avq_mode, push_mode):
    """The paper's baseline (one thread per vertex) and its per-sweep full scan
    of the active vertices give exactly the oracle's results too."""
    graphs = [W.bipartite(3000, 2000, 40000, 2.1, 11), W.random_graph(2000, 16000, 1, 100, 21),
              W.from_arcs(5002, [(0, 2 + i, 1 + i % 9) for i in range(5000)] + [(2 + i, 1, 1 + (i * 31) % 7)
                                                                                for i in range(5000)], 0, 1, "star")]
    graphs += [W.multigraph(int(v), int(6 * v), cmax=25, seed=300 + int(v)) for v in (2, 7, 33, 120)]
    solver.set_options(lanes_per_vertex=lanes, avq_mode=avq_mode, push_mode=push_mode, **WATCHDOG)
    try:
        for g in graphs:
            say(f"[tc/scan] lanes={lanes} avq={avq_mode} push={push_mode} {g.name}")
            check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**WATCHDOG)


@pytest.mark.parametrize("seed", range(30))
def test_paper_single_push_mode(solver, seed):
    """Algorithms 1-2 as printed: one push to the minimum-height neighbour per visit."""
    rng = np.random.default_rng(100 + seed)
    V = int(rng.integers(2, 60))
    g = W.multigraph(V, int(rng.integers(0, 8 * V)), cmax=int(rng.integers(0, 40)), seed=7000 + seed)
    say(f"[paper-mode] seed={seed} V={V}")
    solver.set_options(push_mode=1, **WATCHDOG)
    try:
        check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**WATCHDOG)


@pytest.mark.parametrize("K", [1, 3, 64])
def test_global_relabel_frequency(solver, K):
    g = W.random_graph(2000, 16000, 1, 100, 21)
    say(f"[gr] K={K}")
    solver.set_options(gr_every_sweeps=K, **WATCHDOG)
    try:
        check_against_oracle(g, solver.solve(g))
    finally:
        solver.set_options(**WATCHDOG)


def test_value_only_and_repeatability(solver):
    g = W.config_plain()
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    sides = set()
    for rep in range(5):
        say(f"[repeat] {rep}")
        r = solver.solve(g, want_flow=(rep % 2 == 0), want_side=True)
        check_against_oracle(g, r, ref)
        sides.add(hashlib.sha256(r.side.tobytes()).hexdigest())
    assert len(sides) == 1
    r = solver.solve(g, want_flow=False, want_side=False)
    assert r.value == ref[0]


def test_error_paths(solver):
    from paper_2404_00270_amd import wbpr

    g = W.config_plain()
    ctx = solver.ctx
    rc = wbpr.wbpr_solve(ctx, g.V, g.row_ptr, g.col, g.cap, 5, 5, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    rc = wbpr.wbpr_solve(ctx, g.V, g.row_ptr, g.col, g.cap, 0, g.V, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    bad = g.col.copy()
    bad[17] = g.V + 3  # detected on the device
    rc = wbpr.wbpr_solve(ctx, g.V, g.row_ptr, bad, g.cap, g.s, g.t, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    neg = g.cap.copy()
    neg[5] = -1
    rc = wbpr.wbpr_solve(ctx, g.V, g.row_ptr, g.col, neg, g.s, g.t, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    rp = g.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]
    if rp[10] != rp[11]:
        rc = wbpr.wbpr_solve(ctx, g.V, rp, g.col, g.cap, g.s, g.t, return_code=True)
        assert rc == wbpr.WBPR_EINVAL
    ovf = W.from_arcs(3, [(0, 1, 2**31 - 1), (1, 0, 5), (1, 2, 4)], 0, 2)
    rc = wbpr.wbpr_solve(ctx, ovf.V, ovf.row_ptr, ovf.col, ovf.cap, 0, 2, return_code=True)
    assert rc == wbpr.WBPR_EOVERFLOW
    # parallel arcs whose sum alone leaves int32; a pair summing to 2^31
    for arcs in ([(0, 1, 2**31 - 1), (0, 1, 1), (1, 2, 4)], [(0, 1, 2**30), (1, 0, 2**30), (1, 2, 4)]):
        o = W.from_arcs(3, arcs, 0, 2)
        rc = wbpr.wbpr_solve(ctx, o.V, o.row_ptr, o.col, o.cap, 0, 2, return_code=True)
        assert rc == wbpr.WBPR_EOVERFLOW, arcs
    # largest pair sum that fits: solves
    fit = W.from_arcs(3, [(0, 1, 2**30), (1, 0, 2**30 - 1), (1, 2, 4), (0, 1, 0)], 0, 2)
    check_against_oracle(fit, solver.solve(fit))
    # the context still works after errors
    check_against_oracle(g, solver.solve(g))


def test_device_resident_path_torch(solver):
    import torch

    g = W.random_graph(5000, 40000, 1, 100, 31)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    cap = torch.from_numpy(g.cap).to(dev)
    value = torch.zeros(1, dtype=torch.int64, device=dev)
    flow = torch.zeros(g.E, dtype=torch.int32, device=dev)
    side = torch.zeros(g.V, dtype=torch.uint8, device=dev)
    solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
    torch.cuda.synchronize()

    class R:
        pass

    r = R()
    r.value, r.flow, r.side = int(value.item()), flow.cpu().numpy(), side.cpu().numpy()
    check_against_oracle(g, r)


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["plain", "bipartite", "grid", "rmat"])
def test_full_size_workloads(solver, name):
    gold = _golden()[name]
    say(f"[full] generating {name}")
    g = W.WORKLOADS[name]()
    assert g.sha256() == gold["graph_sha256"], "workload generator drifted"
    say(f"[full] solving {name} V={g.V} E={g.E}")
    r = solver.solve(g)
    say(f"[full] {name} value={r.value} stats={ {k: r.stats[k] for k in ('sweeps', 'global_relabels', 'ms_total')} }")
    assert r.value == gold["value"]
    assert int(r.side.sum()) == gold["sink_side_size"]
    assert hashlib.sha256(r.side.tobytes()).hexdigest() == gold["sink_side_sha256"]
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
    assert c.feasible and c.value == gold["value"] and c.cut_capacity == gold["cut_capacity"]
    assert np.array_equal(c.side, r.side)
