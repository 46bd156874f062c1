"""The batched stream at its stated scale: 4,096 independent instances
(V log-uniform in [256, 65,536], 8V distinct uniform arcs, capacities
U[1,100], s = 0, t = V - 1), about 48M vertices and 386M arcs in all.

Every instance is compared with the oracle's stored answer
(tests/golden/batch_stream_values.txt, written by make_golden.py from the
oracle alone): the value, and the canonical sink side by its size and hash.
Per-arc flows pass the oracle's certificate on every instance with
V > 16,384 and on every 16th of the others.  Two routes:

* batched device solves (wbpr_solve_batch_device) over consecutive groups of
  256 instances, each group one disjoint-union residual graph;
* the continuous-batching server under the default 1 GiB HBM budget, with
  all 4,096 requests queued at once, so admission by footprint decides what
  runs together and results land in a mix unlike the batched groups'.
"""
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_stream_values.txt")
N = 4096
GROUP = 256


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load_golden():
    rows, inputs_sha = {}, None
    with open(GOLDEN) as f:
        for ln in f:
            if ln.startswith("# inputs_sha256"):
                inputs_sha = ln.split()[2]
            if ln.startswith("#") or not ln.strip():
                continue
            i, V, E, value, ssize, shash = ln.split()
            rows[int(i)] = (int(V), int(E), int(value), int(ssize), shash)
    return rows, inputs_sha


@pytest.fixture(scope="module")
def stream():
    t0 = time.time()
    with ThreadPoolExecutor(16) as ex:  # the generator releases the GIL
        gs = list(ex.map(W.batch_instance, range(N)))
    golden, inputs_sha = _load_golden()
    h = hashlib.sha256()
    for g in gs:
        h.update(bytes.fromhex(g.sha256()))
    assert h.hexdigest() == inputs_sha, "generator output changed since the golden file was written"
    say(f"[stream] {N} instances, sum V {sum(g.V for g in gs)}, sum E {sum(g.E for g in gs)}, "
        f"generated in {time.time() - t0:.1f}s")
    return gs, golden


def _side_ok(side, want):
    return int(side.sum()) == want[3] and hashlib.sha256(np.ascontiguousarray(side).tobytes()).hexdigest()[:16] == want[4]


def _certify(g, flow, value):
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, flow)
    assert c.feasible, (g.name, c.code, c.bad)
    assert c.value == value and c.cut_capacity == value, g.name


def _needs_certificate(i, g):
    return g.V > 16384 or i % 16 == 0


def test_stream_batched_groups(stream):
    import torch

    from paper_2404_00270_amd import wbpr

    gs, golden = stream
    dev = torch.device("cuda:0")
    t_solve = 0.0
    certified = 0
    with wbpr.Solver(0, max_wall_ms=120_000) as solver:
        for g0 in range(0, N, GROUP):
            grp = gs[g0:g0 + GROUP]
            say(f"[stream-batch] instances {g0}..{g0 + len(grp) - 1} V={sum(g.V for g in grp)} "
                f"E={sum(g.E for g in grp)}")
            rp = torch.from_numpy(np.concatenate([g.row_ptr for g in grp])).to(dev)
            col = torch.from_numpy(np.concatenate([g.col for g in grp])).to(dev)
            cap = torch.from_numpy(np.concatenate([g.cap for g in grp])).to(dev)
            Et = int(col.shape[0])
            values = torch.zeros(len(grp), dtype=torch.int64, device=dev)
            flows = torch.zeros(Et, dtype=torch.int32, device=dev)
            sides = torch.zeros(sum(g.V for g in grp), dtype=torch.uint8, device=dev)
            stream_h = torch.cuda.current_stream(dev).cuda_stream
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            wbpr.wbpr_solve_batch_device(solver.ctx, [g.V for g in grp], [g.E for g in grp], [g.s for g in grp],
                                         [g.t for g in grp], rp.data_ptr(), col.data_ptr(), cap.data_ptr(), stream_h,
                                         values.data_ptr(), flows.data_ptr(), sides.data_ptr())
            t_solve += time.perf_counter() - t0
            vals = values.cpu().numpy()
            fl = flows.cpu().numpy()
            sd = sides.cpu().numpy()
            vo = eo = 0
            for k, g in enumerate(grp):
                i = g0 + k
                want = golden[i]
                assert (g.V, g.E) == want[:2], i
                assert int(vals[k]) == want[2], (i, int(vals[k]), want[2])
                assert _side_ok(sd[vo:vo + g.V], want), i
                if _needs_certificate(i, g):
                    _certify(g, fl[eo:eo + g.E], want[2])
                    certified += 1
                vo += g.V
                eo += g.E
    say(f"[stream-batch] {N} instances equal the oracle's; {certified} flows certified; "
        f"batched solve time {t_solve * 1e3:.0f} ms ({N / t_solve:.0f} solves/s)")


def test_stream_served_under_budget(stream):
    from paper_2404_00270_amd import wbpr

    gs, golden = stream
    certified = 0
    with wbpr.Solver(0, max_wall_ms=120_000) as solver:
        with wbpr.Server(solver, hbm_budget_bytes=1 << 30, want_flows=True, want_sides=True) as srv:
            t0 = time.perf_counter()
            tickets = [srv.submit(g) for g in gs]
            say(f"[stream-served] {N} requests queued in {time.perf_counter() - t0:.2f}s")
            for i, (g, tk) in enumerate(zip(gs, tickets)):
                r = srv.wait(tk, 120_000)
                assert r is not None and r.status == 0, (i, None if r is None else r.status)
                want = golden[i]
                assert r.value == want[2], (i, r.value, want[2])
                assert _side_ok(r.side, want), i
                if _needs_certificate(i, g):
                    _certify(g, r.flow, want[2])
                    certified += 1
            st = srv.stats()
    say(f"[stream-served] {N} results equal the oracle's; {certified} flows certified; "
        f"{st['solves_per_s']:.0f} solves/s, p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
        f"peak resident {st['peak_resident']}")
