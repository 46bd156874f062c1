"""GPU tests of the continuous-batching server.

Every served result must be exactly what the instance gives alone (a plain
solve on its own context, and the oracle): value, canonical cut side, and a
per-arc flow that passes the oracle's certificate.  Requests are submitted
from several threads at staggered times, so later ones join rounds that
earlier ones are already in; a small HBM budget forces admission to wait for
space.
"""
import sys
import threading
import time

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


def _stream(n, seed, vmax=8192):
    rng = np.random.default_rng(seed)
    gs = []
    for i in range(n):
        if i % 4 == 3:
            V = int(rng.integers(2, 40))
            gs.append(W.multigraph(V, int(rng.integers(0, 6 * V)), cmax=int(rng.integers(0, 30)),
                                   seed=70_000 + 1000 * seed + i))
        else:
            gs.append(W.batch_instance(1000 * seed + i, vmin=64, vmax=vmax))
    return gs


def _check(g, r, alone=None):
    value, side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    assert r.status == 0, (g.name, r.status)
    assert r.value == value, (g.name, r.value, value)
    if alone is not None:
        assert r.value == alone.value
        assert np.array_equal(r.side, alone.side)
    if r.side is not None:
        assert np.array_equal(r.side, side), g.name
    if r.flow is not None:
        c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, r.flow)
        assert c.feasible and c.value == value and c.cut_capacity == value, (g.name, c.code, c.bad)


def test_served_results_equal_alone(solver):
    from paper_2404_00270_amd import wbpr

    gs = _stream(40, 1)
    alone = [solver.solve(g) for g in gs]
    with wbpr.Server(solver, hbm_budget_bytes=256 << 20, max_slots=64) as srv:
        tickets = [None] * len(gs)

        def client(k):
            for i in range(k, len(gs), 4):
                tickets[i] = srv.submit(gs[i])
                time.sleep(0.002 * (i % 3))

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        say(f"[server] submitted {len(gs)}")
        res = [srv.wait(tk, 120_000) for tk in tickets]
        st = srv.stats()
    say(f"[server] stats {st}")
    for g, r, a in zip(gs, res, alone):
        assert r is not None, g.name
        _check(g, r, a)
    assert st["completed"] == len(gs) and st["failed"] == 0
    assert st["peak_resident"] > 1, "requests never overlapped on the device"
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_tight_budget_queues_and_stays_exact(solver):
    from paper_2404_00270_amd import wbpr

    gs = _stream(24, 2, vmax=16384)
    with wbpr.Server(solver, hbm_budget_bytes=48 << 20, max_slots=8) as srv:
        st0 = srv.stats()
        say(f"[server-tight] Vcap={st0['Vcap']} Ecap={st0['Ecap']}")
        tickets = []
        for g in gs:
            rc, tk = srv.submit(g, return_code=True)
            if rc == wbpr.WBPR_ETOOBIG:
                assert g.V > st0["Vcap"] // 2 or g.E > st0["Ecap"] // 2
                tickets.append(None)
                continue
            assert rc == 0
            tickets.append(tk)
        res = [srv.wait(tk, 120_000) if tk is not None else None for tk in tickets]
        st = srv.stats()
    say(f"[server-tight] stats {st}")
    assert st["peak_resident"] <= 8
    for g, r in zip(gs, res):
        if r is not None:
            _check(g, r)
    assert sum(r is not None for r in res) >= len(gs) // 2


def test_value_only_server_and_poll(solver):
    from paper_2404_00270_amd import wbpr

    gs = _stream(10, 3)
    with wbpr.Server(solver, hbm_budget_bytes=128 << 20, want_flows=False, want_sides=False) as srv:
        tks = [srv.submit(g) for g in gs]
        out = {}
        t0 = time.time()
        while len(out) < len(tks) and time.time() - t0 < 120:
            for tk in tks:
                if tk not in out:
                    r = srv.poll(tk)
                    if r is not None:
                        out[tk] = r
            time.sleep(0.001)
    for g, tk in zip(gs, tks):
        r = out[tk]
        assert r.flow is None and r.side is None
        assert r.value == oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)[0]


def test_server_rejections_and_shutdown(solver):
    from paper_2404_00270_amd import wbpr

    srv = wbpr.Server(solver, hbm_budget_bytes=32 << 20, max_slots=4)
    st = srv.stats()
    big = W.random_graph(int(st["Vcap"]), 4 * int(st["Vcap"]), 1, 10, 3)
    rc, _ = srv.submit(big, return_code=True)
    assert rc == wbpr.WBPR_ETOOBIG
    g = W.config_plain()
    bad = W.Graph(g.V, g.row_ptr, np.where(np.arange(g.E) == 7, g.V, g.col).astype(np.int32), g.cap, g.s, g.t)
    rc, _ = srv.submit(bad, return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    rc, _ = srv.submit(W.Graph(g.V, g.row_ptr, g.col, g.cap, 3, 3), return_code=True)
    assert rc == wbpr.WBPR_EINVAL
    with pytest.raises(wbpr.WbprError):
        srv.poll(123456)
    # overflowing merged capacity is found on the device, alone in its group
    ovf = W.from_arcs(3, [(0, 1, 2**31 - 1), (1, 0, 5), (1, 2, 4)], 0, 2)
    tk_ovf = srv.submit(ovf)
    tk_ok = srv.submit(g)
    r = srv.wait(tk_ovf, 60_000)
    assert r.status == wbpr.WBPR_EOVERFLOW
    _check(g, srv.wait(tk_ok, 60_000))
    # destroy with requests in flight returns promptly
    for i in range(6):
        srv.submit(W.batch_instance(i, vmin=64, vmax=4096))
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 60


@pytest.mark.parametrize("batch_kernel", [1, 2])
def test_server_modes_equal_alone(batch_kernel):
    """Both ways the server solves: rounds of shared launches (the default)
    and the persistent kernel with live admission (batch_kernel 2, for every
    eligible request); requests from several threads, staggered."""
    from paper_2404_00270_amd import wbpr

    gs = _stream(32, 7, vmax=32768)
    with wbpr.Solver(0, batch_kernel=batch_kernel, **WATCHDOG) as s:
        alone = [s.solve(g) for g in gs]
        with wbpr.Server(s, hbm_budget_bytes=256 << 20, max_slots=64) as srv:
            tickets = [None] * len(gs)

            def client(k):
                for i in range(k, len(gs), 4):
                    tickets[i] = srv.submit(gs[i])
                    time.sleep(0.003 * (i % 4))

            th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
            for t in th:
                t.start()
            for t in th:
                t.join()
            res = [srv.wait(tk, 120_000) for tk in tickets]
            st = srv.stats()
    say(f"[server-mode {batch_kernel}] rounds={st['rounds']} solves/s={st['solves_per_s']:.0f} "
        f"p50={st['p50_ms']:.2f} p99={st['p99_ms']:.2f} peak_resident={st['peak_resident']}")
    for g, r, a in zip(gs, res, alone):
        assert r is not None, g.name
        _check(g, r, a)
    if batch_kernel == 2:
        assert st["rounds"] == 0  # every request was eligible: no round ran
    else:
        assert st["rounds"] > 0


def test_server_persistent_and_rounds_together():
    """A request too large for the persistent kernel (more than 131,072
    vertices) is solved by the rounds while the others go through the
    kernel; every result equals the oracle's."""
    from paper_2404_00270_amd import wbpr

    big = W.random_graph(140_000, 700_000, 1, 100, 71)
    gs = _stream(12, 8, vmax=8192)
    gs.insert(5, big)
    with wbpr.Solver(0, batch_kernel=2, **WATCHDOG) as solver, \
            wbpr.Server(solver, hbm_budget_bytes=512 << 20, max_slots=32) as srv:
        tickets = [srv.submit(g) for g in gs]
        res = [srv.wait(tk, 120_000) for tk in tickets]
        st = srv.stats()
    say(f"[server-mixed] rounds={st['rounds']} completed={st['completed']}")
    for g, r in zip(gs, res):
        assert r is not None, g.name
        _check(g, r)
    assert st["rounds"] > 0
