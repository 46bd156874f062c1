"""GPU parity of batched solves: many instances resident in one arena, solved
by shared sweeps and one multi-root global relabel per round.

Every instance of a batch must give exactly what the oracle gives for it
alone (value, canonical sink side, a certified per-arc flow), whatever the
mix of sizes, the sweep batching (captured graph or direct launches, fixed or
adaptive relabel frequency) and the outputs asked for.
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


@pytest.fixture(scope="module")
def solver():
    from paper_2404_00270_amd import wbpr

    s = wbpr.Solver(0, **WATCHDOG)
    yield s
    s.close()


def _mixed_batch(seed, n_small=12, n_stream=6, vmax=4096):
    rng = np.random.default_rng(seed)
    gs = []
    for i in range(n_small):
        V = int(rng.integers(2, 50))
        gs.append(W.multigraph(V, int(rng.integers(0, 6 * V)), cmax=int(rng.integers(0, 30)),
                               seed=90_000 + 100 * seed + i))
    for i in range(n_stream):
        gs.append(W.batch_instance(7 * seed + i, vmin=64, vmax=vmax))
    gs.append(W.from_arcs(2, [], 0, 1, "no-arcs"))
    gs.append(W.from_arcs(4, [(1, 2, 5), (2, 3, 5)], 0, 3, "source-isolated"))
    order = rng.permutation(len(gs))
    return [gs[k] for k in order]


def _check_batch(gs, res, refs=None):
    for i, g in enumerate(gs):
        value, side, cutcap = refs[i] if refs else oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
        assert res.values[i] == value, (i, g.name, int(res.values[i]), value)
        if res.sides is not None:
            assert np.array_equal(res.sides[i], side), (i, g.name)
        if res.flows is not None:
            c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, res.flows[i])
            assert c.feasible, (i, g.name, c.code, c.bad)
            assert c.value == value and c.cut_capacity == value
            assert np.array_equal(c.side, side)


@pytest.mark.parametrize("seed", range(4))
def test_mixed_batch_matches_oracle(solver, seed):
    gs = _mixed_batch(seed)
    say(f"[batch] seed={seed} n={len(gs)} V={sum(g.V for g in gs)} E={sum(g.E for g in gs)}")
    res = solver.solve_batch(gs)
    assert res.stats["instances"] == len(gs)
    _check_batch(gs, res)


def test_batch_of_small_instances_in_lds(solver):
    """A batch of instances that all fit one workgroup's LDS, alone on the
    device, is solved whole by one workgroup each (no rounds)."""
    rng = np.random.default_rng(5)
    gs = [W.multigraph(int(rng.integers(2, 60)), int(rng.integers(0, 300)), cmax=25, seed=600 + i) for i in range(20)]
    gs += [W.batch_instance(100 + i, vmin=64, vmax=900) for i in range(12)]
    say(f"[batch-lds] n={len(gs)}")
    res = solver.solve_batch(gs)
    assert res.stats["lds_solved"] == len(gs)
    _check_batch(gs, res)
    # with one larger instance the group takes the rounds
    res = solver.solve_batch(gs + [W.batch_instance(7, vmin=2048, vmax=4096)])
    assert res.stats["lds_solved"] == 0
    _check_batch(gs + [W.batch_instance(7, vmin=2048, vmax=4096)], res)


def test_batch_outputs_subsets(solver):
    gs = _mixed_batch(11)
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    for wf, ws in ((False, False), (False, True), (True, False)):
        say(f"[batch-out] flows={wf} sides={ws}")
        res = solver.solve_batch(gs, want_flow=wf, want_side=ws)
        assert (res.flows is None) == (not wf) and (res.sides is None) == (not ws)
        _check_batch(gs, res, refs)


@pytest.mark.parametrize("opts", [
    dict(no_graph=1),
    dict(gr_every_sweeps=3),
    dict(gr_every_sweeps=1, no_graph=1),
    dict(gr_work_permille=1),
    dict(gr_work_permille=20, push_mode=1),
    dict(time_kernels=1),
    dict(lanes_per_vertex=4, split_degree=3, block_degree=9),
])
def test_batch_launch_variants(solver, opts):
    gs = _mixed_batch(21, n_small=6, n_stream=4)
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    say(f"[batch-variant] {opts}")
    solver.set_options(**opts, **WATCHDOG)
    try:
        _check_batch(gs, solver.solve_batch(gs), refs)
    finally:
        solver.set_options(**WATCHDOG)


@pytest.mark.parametrize("permille", [1, 30, 1000])
def test_single_solve_relabel_budget(solver, permille):
    """Early halts of the sweep batch (tiny relabel budget) keep parity."""
    g = W.random_graph(4000, 40000, 1, 100, 41)
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    say(f"[budget] permille={permille}")
    for no_graph in (0, 1):
        solver.set_options(gr_work_permille=permille, no_graph=no_graph, **WATCHDOG)
        try:
            r = solver.solve(g)
        finally:
            solver.set_options(**WATCHDOG)
        assert r.value == ref[0]
        assert np.array_equal(r.side, ref[1])
        c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
        assert c.feasible and c.value == ref[0]


def test_batch_of_one_equals_single(solver):
    g = W.batch_instance(3)
    a = solver.solve(g)
    b = solver.solve_batch([g])
    assert a.value == int(b.values[0])
    assert np.array_equal(a.side, b.sides[0])


def test_back_to_back_batches_reuse_arena(solver):
    """A larger batch, then a smaller one, then a single solve on one context."""
    big = _mixed_batch(31, n_small=8, n_stream=8, vmax=8192)
    small = _mixed_batch(32, n_small=3, n_stream=1)
    for gs in (big, small):
        say(f"[reuse] n={len(gs)}")
        _check_batch(gs, solver.solve_batch(gs))
    g = W.config_plain()
    r = solver.solve(g)
    assert r.value == oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)[0]


def test_batch_bad_instance_rejected(solver):
    from paper_2404_00270_amd import wbpr

    gs = _mixed_batch(41, n_small=4, n_stream=2)
    bad = gs[2]
    if bad.E == 0:
        bad = gs[3] if gs[3].E else W.multigraph(10, 30, seed=5)
        gs[2] = bad
    col = bad.col.copy()
    col[0] = bad.V  # out of range for its own instance, in range for the union
    gs_bad = list(gs)
    gs_bad[2] = W.Graph(bad.V, bad.row_ptr, col, bad.cap, bad.s, bad.t, "bad-col")
    rc = wbpr.wbpr_solve_batch(solver.ctx, gs_bad, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    gs_st = list(gs)
    gs_st[1] = W.Graph(gs[1].V, gs[1].row_ptr, gs[1].col, gs[1].cap, 0, 0, "s==t")
    rc = wbpr.wbpr_solve_batch(solver.ctx, gs_st, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    _check_batch(gs, solver.solve_batch(gs))


def _faulty(gs):
    """Copies of valid instances with one defect each, and the code each must get."""
    from paper_2404_00270_amd import wbpr

    b = gs[0] if gs[0].E else W.multigraph(10, 30, seed=5)
    col = b.col.copy()
    col[0] = b.V  # in range for the union of the batch, not for its own instance
    cap = b.cap.copy()
    cap[-1] = -3
    return [
        (W.Graph(b.V, b.row_ptr, col, b.cap, b.s, b.t, "bad-col"), wbpr.WBPR_EINVAL),
        (W.Graph(b.V, b.row_ptr, b.col, b.cap, b.s, b.s, "s==t"), wbpr.WBPR_EINVAL),
        (W.Graph(b.V, b.row_ptr, b.col, cap, b.s, b.t, "negative-cap"), wbpr.WBPR_EINVAL),
        (W.from_arcs(3, [(0, 1, 2**31 - 1), (1, 0, 5), (1, 2, 4)], 0, 2, "overflow"), wbpr.WBPR_EOVERFLOW),
    ]


def test_batch_per_instance_status(solver):
    good = _mixed_batch(43, n_small=4, n_stream=3)
    bad = _faulty(good)
    mixed = list(good)
    for k, (g, _) in enumerate(bad):
        mixed.insert(2 * k + 1, g)
    codes = {id(g): c for g, c in bad}
    say(f"[batch-status] n={len(mixed)}")
    res = solver.solve_batch(mixed, per_instance=True)
    for i, g in enumerate(mixed):
        if id(g) in codes:
            assert res.status[i] == codes[id(g)], (g.name, res.status[i])
            assert res.values[i] == 0
        else:
            assert res.status[i] == 0, (g.name, res.status[i])
            value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
            assert res.values[i] == value and np.array_equal(res.sides[i], side), g.name
            c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, res.flows[i])
            assert c.feasible and c.value == value
    # all valid: one group, every status 0
    res = solver.solve_batch(good, per_instance=True)
    assert (res.status == 0).all()
    _check_batch(good, res)


def test_batch_device_per_instance_status(solver):
    import torch

    from paper_2404_00270_amd import wbpr

    good = _mixed_batch(44, n_small=3, n_stream=2)
    bad = _faulty(good)
    gs = [good[0], bad[0][0], good[1], bad[3][0]] + good[2:]
    want = [0, wbpr.WBPR_EINVAL, 0, wbpr.WBPR_EOVERFLOW] + [0] * (len(good) - 2)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(np.concatenate([g.row_ptr for g in gs]).astype(np.int64)).to(dev)
    col = torch.from_numpy(np.concatenate([g.col for g in gs]).astype(np.int32)).to(dev)
    cap = torch.from_numpy(np.concatenate([g.cap for g in gs]).astype(np.int32)).to(dev)
    n = len(gs)
    values = torch.zeros(n, dtype=torch.int64, device=dev)
    sides = torch.zeros(sum(g.V for g in gs), dtype=torch.uint8, device=dev)
    status = np.full(n, -1, np.int32)
    torch.cuda.synchronize()
    wbpr.wbpr_solve_batch_device(solver.ctx, [g.V for g in gs], [g.E for g in gs], [g.s for g in gs],
                                 [g.t for g in gs], rp.data_ptr(), col.data_ptr(), cap.data_ptr(), 0,
                                 values.data_ptr(), 0, sides.data_ptr(), status=status)
    torch.cuda.synchronize()
    assert status.tolist() == want
    hv, hs = values.cpu().numpy(), sides.cpu().numpy()
    vo = np.cumsum([0] + [g.V for g in gs])
    for i, g in enumerate(gs):
        if want[i] == 0:
            value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
            assert hv[i] == value and np.array_equal(hs[vo[i]:vo[i + 1]], side), g.name
        else:
            assert hv[i] == 0


def test_batch_device_packed_torch(solver):
    import torch

    from paper_2404_00270_amd import wbpr

    gs = _mixed_batch(51, n_small=5, n_stream=3)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(np.concatenate([g.row_ptr for g in gs]).astype(np.int64)).to(dev)
    col = torch.from_numpy(np.concatenate([g.col for g in gs]).astype(np.int32)).to(dev)
    cap = torch.from_numpy(np.concatenate([g.cap for g in gs]).astype(np.int32)).to(dev)
    n = len(gs)
    values = torch.zeros(n, dtype=torch.int64, device=dev)
    flows = torch.zeros(max(1, sum(g.E for g in gs)), dtype=torch.int32, device=dev)
    sides = torch.zeros(sum(g.V for g in gs), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    wbpr.wbpr_solve_batch_device(solver.ctx, [g.V for g in gs], [g.E for g in gs], [g.s for g in gs],
                                 [g.t for g in gs], rp.data_ptr(), col.data_ptr(), cap.data_ptr(), 0,
                                 values.data_ptr(), flows.data_ptr(), sides.data_ptr())
    torch.cuda.synchronize()
    hv, hf, hs = values.cpu().numpy(), flows.cpu().numpy(), sides.cpu().numpy()

    class R:
        pass

    r = R()
    r.values = hv
    eo = np.cumsum([0] + [g.E for g in gs])
    vo = np.cumsum([0] + [g.V for g in gs])
    r.flows = [hf[eo[i]:eo[i + 1]] for i in range(n)]
    r.sides = [hs[vo[i]:vo[i + 1]] for i in range(n)]
    _check_batch(gs, r)


def test_uploaded_graph_many_pairs(solver):
    """One residual build, many (s, t) solves: each equals the oracle's."""
    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(77)
    for g0 in (W.random_graph(3000, 24000, 1, 100, 61), W.bipartite(2000, 1500, 20000, 2.1, 62),
               W.multigraph(40, 200, cmax=20, seed=63)):
        with wbpr.UploadedGraph(solver, g0) as ug:
            pairs = [(g0.s, g0.t)] + [tuple(int(x) for x in rng.choice(g0.V, 2, replace=False)) for _ in range(6)]
            for s_, t_ in pairs:
                g = W.Graph(g0.V, g0.row_ptr, g0.col, g0.cap, s_, t_, f"{g0.name}[{s_}->{t_}]")
                say(f"[uploaded] {g.name}")
                wf = (s_ + t_) % 2 == 0
                r = ug.solve(s_, t_, want_flow=wf)
                value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, s_, t_)
                assert r.value == value, (g.name, r.value, value)
                assert np.array_equal(r.side, side)
                if wf:
                    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, s_, t_, r.flow)
                    assert c.feasible and c.value == value
            assert ug.solve(0, 0, return_code=True) == wbpr.WBPR_EINVAL
            assert ug.solve(0, g0.V, return_code=True) == wbpr.WBPR_EINVAL
            r = ug.solve(g0.s, g0.t)  # still usable after rejected calls
            assert r.value == oracle.reference(g0.V, g0.row_ptr, g0.col, g0.cap, g0.s, g0.t)[0]


def test_autotune_then_tuned_solves(solver):
    """The autotuner returns a schedule; later automatic solves of that shape use it, exactly."""
    from paper_2404_00270_amd import wbpr

    g = W.random_graph(6000, 48000, 1, 100, 71)
    ref = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    with wbpr.Solver(0, **WATCHDOG) as s2:
        best, ms = s2.autotune(g, max_trials=6, include_full_scan=True)
        say(f"[autotune] best={best} ms={ms:.2f}")
        assert best["lanes_per_vertex"] in (4, 8, 16, 32) and best["gr_work_permille"] > 0 and ms > 0
        g2 = W.random_graph(6000, 48000, 1, 100, 72)  # same shape class
        r = s2.solve(g2)
        assert r.stats["lanes_per_vertex"] == best["lanes_per_vertex"]
        assert r.value == oracle.reference(g2.V, g2.row_ptr, g2.col, g2.cap, g2.s, g2.t)[0]
        r = s2.solve(g)
        assert r.value == ref[0] and np.array_equal(r.side, ref[1])


@pytest.mark.parametrize("layout", [1, 2])
def test_persistent_per_instance_kernel(layout):
    """Every instance of a mixed batch solved by the persistent kernel (one
    workgroup per instance, claimed largest first): results equal the
    oracle's, flows certified, in both residual layouts."""
    from paper_2404_00270_amd import wbpr

    gs = _mixed_batch(31, n_small=10, n_stream=24, vmax=65536)
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    with wbpr.Solver(0, batch_kernel=2, layout=layout, **WATCHDOG) as s:
        say(f"[wg] layout={layout} n={len(gs)} V={sum(g.V for g in gs)} E={sum(g.E for g in gs)}")
        res = s.solve_batch(gs)
        say(f"[wg] wg_solved={res.stats['wg_solved']} fallbacks={res.stats['wg_fallbacks']} "
            f"lds={res.stats['lds_solved']} sweeps={res.stats['sweeps']}")
        assert res.stats["wg_solved"] + res.stats["wg_fallbacks"] + res.stats["lds_solved"] == len(gs)
        assert res.stats["wg_solved"] > 0
        _check_batch(gs, res, refs)
        for wf, ws in ((False, True), (False, False)):  # value only, and value with sides
            r2 = s.solve_batch(gs, want_flow=wf, want_side=ws)
            _check_batch(gs, r2, refs)


@pytest.mark.parametrize("cap", ["1", "2"])
def test_persistent_kernel_hands_over_to_rounds(monkeypatch, cap):
    """Instances stopped at the persistent kernel's round cap (forced low from
    the host) are finished by the rounds of launches: same results."""
    from paper_2404_00270_amd import wbpr

    monkeypatch.setenv("WBPR_WG_ROUND_CAP", cap)
    gs = [W.batch_instance(200 + i, vmin=256, vmax=8192) for i in range(12)]
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    with wbpr.Solver(0, batch_kernel=2, **WATCHDOG) as s:
        res = s.solve_batch(gs)
        say(f"[wg-cap {cap}] wg_solved={res.stats['wg_solved']} fallbacks={res.stats['wg_fallbacks']}")
        assert res.stats["wg_solved"] + res.stats["wg_fallbacks"] == len(gs)
        if cap == "1":  # one BFS round is too few for any of them
            assert res.stats["wg_fallbacks"] > 0
        _check_batch(gs, res, refs)
