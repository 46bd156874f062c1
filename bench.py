"""Benchmark: one full max-flow solve per step on one MI355X.

A step is the whole hot path on one synthetic graph already resident in HBM:
residual-graph build (bidirectional CSR), preflow, vertex-centric push-relabel
sweeps with on-GPU global relabels until no active vertex can reach the sink,
the canonical min-cut side, the second phase that returns stranded excess to
the source, and the per-arc flow decode.  The default workload is the R-MAT
scale-22 graph (4,194,304 vertices, edge factor 16, a/b/c/d =
.57/.19/.19/.05, duplicates and self-loops removed, capacities U[1,1000],
s = max out-degree, t = max in-degree vertex other than s), the synthetic
stand-in for the paper's large social-network max-flow inputs.

Prints ONE JSON line.  value = arc-scans per second over the whole timed
solve (residual entries examined by the sweeps / wall time); ms_per_step is
the solve time.  The timed steps run exactly as a caller would (sweep
batches replayed as captured hipGraphs, no events).

"roofline" prices the push-relabel sweep, the path's hot loop: the three
sweep kernels (short-row tiles, one wave per medium row, workgroup chunks
of long rows) together, their algorithmic bytes over their device time.
Durations come from HIP events recorded on the library's stream around
every launch of an extra instrumented solve of the same graph, run right
after the timed region (events cannot sit between the kernels of a captured
batch).  "secondary" prices the global relabel and the residual-graph
builder the same way, and "kernels" lists every kernel.

"workloads" solves the other three configurations (plain 1k-vertex graph,
50k+50k Zipf bipartite matching, 2048x2048 grid cut) and checks each value
against the oracle's stored answer; "rcsr_ms" is the headline graph in the
paper's other residual layout.  "stream" is the batched and served stream
as configured: 4,096 instances (V log-uniform in [256, 65536], out-degree 8,
capacities U[1,100]) solved one at a time, in device batches, through the
continuous-batching server with all of them queued at once, and with
Poisson arrivals at 0.25, 0.5, 1 and 2 times the one-at-a-time rate; every
route's values and cut sides are checked against the one-at-a-time results
and the values against the oracle's stored answers.  "cpu_baseline" times
both CPU oracle solvers (FIFO push-relabel, Dinic; one thread each, run
side by side beside the GPU legs) on the headline graph itself.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (int32 residuals, int64 excesses, int32
# heights):
#   sweep kernels  per arc-scan 12 B (BCSR, RCSR forward entry): entry
#                  {column, residual} 8 B + height of the column 4 B (an RCSR
#                  reverse entry adds its 4 B flow gather: 16 B, counted as
#                  12 B here, so RCSR figures are a lower bound); per queued
#                  vertex 24 B: queue slot 4 + row bounds 8 + e(u) 8 + h(u) 4;
#                  per push 52 B: two residual atomics (2 x 8 B read+write),
#                  two excess atomics (2 x 16 B read+write), mate index 4 B;
#                  per relabel 4 B.
#   global relabel per top-down entry 12 B (entry 8 + head height 4); per
#                  bottom-up entry 9 B (entry 8 + visit code 1); per vertex
#                  and launch 17 B (height reset 4 + visit reset 1 + queue
#                  rebuild reads e 8 + h 4).
#   builder (BCSR) reads row_ptr 8 B per vertex and column + capacity 8 B per
#                  arc; writes row bounds 8 B per vertex, 16 B per merged
#                  entry (entry 8, mate 4, merged capacity 4) and 12 B per arc
#                  (entry index, earlier parallel capacity, capacity): the
#                  input once and the output once, no sort traffic.
B_SCAN, B_QUEUED, B_PUSH, B_RELABEL = 12, 24, 52, 4
B_BFS_TD, B_BFS_BU, B_BFS_V = 12, 9, 17
KERNELS = ["k_sweep_tile", "k_sweep_tile<64> (medium rows)", "k_sweep_chunk (long-row chunks)", "k_global_relabel"]
SWEEP_FAMILY = "sweep kernels (k_sweep_tile<P>, k_sweep_tile<64>, k_sweep_chunk*)"


def kernel_bytes(st, k):
    if k < 3:
        return (B_SCAN * st["kernel_arc_scans"][k] + B_QUEUED * st["kernel_queued"][k]
                + B_PUSH * st["kernel_pushes"][k] + B_RELABEL * st["kernel_relabels"][k])
    td = st["bfs_topdown_scans"]
    bu = st["bfs_scans"] - td
    return B_BFS_TD * td + B_BFS_BU * bu + B_BFS_V * st["V"] * st["kernel_launches"][3]


def builder_bytes(st):
    return 16 * st["V"] + 20 * st["E"] + 16 * st["M"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CpuBaseline:
    """Both CPU oracle solvers on one graph, one thread each, side by side in
    the background (the oracle's C code releases the GIL); the faster one is
    the reported baseline."""

    def __init__(self, g):
        self.g = g
        self.res = {}
        self.threads = []

    def start(self):
        import oracle

        def run(name, fn):
            t0 = time.perf_counter()
            r = fn(self.g.V, self.g.row_ptr, self.g.col, self.g.cap, self.g.s, self.g.t)
            self.res[name] = (time.perf_counter() - t0, r.value, r.arc_scans)

        for name, fn in (("fifo_pr", oracle.fifo_pr), ("dinic", oracle.dinic)):
            th = threading.Thread(target=run, args=(name, fn), daemon=True)
            th.start()
            self.threads.append(th)
        return self

    def result(self, gpu_ms, timeout_s=600):
        t_end = time.perf_counter() + timeout_s
        for th in self.threads:
            th.join(max(0.0, t_end - time.perf_counter()))
        if not self.res:
            return None
        name = min(self.res, key=lambda k: self.res[k][0])
        dt, value, scans = self.res[name]
        per = {k: {"solve_s": round(v[0], 2), "value": v[1], "arc_scans": v[2]} for k, v in self.res.items()}
        g = self.g
        return {
            "value": round(dt * 1000.0, 1),
            "unit": "ms per solve",
            "cores": len(self.threads),
            "kind": "oracle",
            "solver": {"fifo_pr": "FIFO push-relabel", "dinic": "Dinic"}[name],
            "sample": f"the headline graph itself ({g.name}, V={g.V}, E={g.E}): both oracle solvers, one "
                      f"thread each, run side by side beside the GPU legs; the faster is reported",
            "solvers": per,
            "same_value_as_gpu": None,
            "host_cpu": host_cpu_model(),
            "host_nproc": os.cpu_count(),
            "gpu_speedup": round(dt * 1000.0 / gpu_ms, 1) if gpu_ms else None,
        }


def kernel_table(stats):
    kernels = []
    for k in range(4):
        ms = sum(st["kernel_ms"][k] for st in stats)
        launches = sum(st["kernel_launches"][k] for st in stats)
        nbytes = sum(kernel_bytes(st, k) for st in stats)
        kernels.append({"kernel": KERNELS[k], "ms": round(ms, 3), "launches": launches,
                        "algorithmic_GB": round(nbytes / 1e9, 4),
                        "GBps": round(nbytes / (ms / 1e3) / 1e9, 2) if ms > 0 else None})
    ms = sum(st["kernel_build_ms"] for st in stats)
    nbytes = sum(builder_bytes(st) for st in stats)
    kernels.append({"kernel": "builder (all build kernels)", "ms": round(ms, 3), "launches": len(stats),
                    "algorithmic_GB": round(nbytes / 1e9, 4),
                    "GBps": round(nbytes / (ms / 1e3) / 1e9, 2) if ms > 0 else None})
    return kernels


def measured_traffic(kernel: str, workload: str):
    """Calibrated HBM bytes (FETCH_SIZE and WRITE_SIZE counters, scaled by
    what they read for a plain device copy) from the committed rocprofv3
    counter runs: per solve for the sweep family and the builder, per launch
    for the global relabel; None when the kernel sources changed since the
    counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in rec["sources"])).hexdigest()
    if h != rec["sources_sha256"]:
        return None
    return rec.get("bytes", {}).get(kernel)


def _priced(name, nbytes, ms, launches, unit_note):
    if ms <= 0 or launches <= 0:
        return None
    achieved = nbytes / (ms / 1e3) / 1e9
    return {
        "kernel": name,
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": None,
        "launches": launches,
        "avg_launch_us": round(ms * 1e3 / launches, 3),
        "algorithmic_bytes_per_launch": round(nbytes / launches, 1),
        "note": unit_note,
    }


def roofline_of(stats, kernels):
    """Headline: the sweep family; secondary: global relabel and builder."""
    n = len(stats)
    sw_bytes = sum(kernel_bytes(st, k) for st in stats for k in range(3))
    sw_ms = sum(kernels[k]["ms"] for k in range(3))
    sw_launches = sum(kernels[k]["launches"] for k in range(3))
    head = _priced(SWEEP_FAMILY, sw_bytes, sw_ms, sw_launches,
                   "achieved = algorithmic bytes of every sweep-kernel launch / their summed event-timed "
                   "durations; traffic = counter bytes of the sweep kernels per solve")
    if head is not None:
        head["per_solve_bytes"] = round(sw_bytes / n, 1)
        head["per_solve_ms"] = round(sw_ms / n, 3)
        head["share_of_kernel_time"] = round(sw_ms / max(1e-9, sum(k["ms"] for k in kernels)), 3)
    rel = _priced(KERNELS[3], sum(kernel_bytes(st, 3) for st in stats), kernels[3]["ms"], kernels[3]["launches"],
                  "per cooperative launch")
    bld = _priced("builder", sum(builder_bytes(st) for st in stats), kernels[4]["ms"], n,
                  "per solve: input read once plus output written once over the builder's device time")
    return head, [x for x in (rel, bld) if x is not None]


def other_workloads(names, dev, steps=3):
    """Solve times of the other configurations, each value checked against
    the oracle's stored answer."""
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    with open(os.path.join(ROOT, "tests", "golden", "workload_values.json")) as f:
        gold = json.load(f)
    out = {}
    for name in names:
        t0 = time.perf_counter()
        g = W.WORKLOADS[name]()
        gen_s = time.perf_counter() - t0
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        cap = torch.from_numpy(g.cap).to(dev)
        value = torch.zeros(1, dtype=torch.int64, device=dev)
        flow = torch.zeros(max(g.E, 1), dtype=torch.int32, device=dev)
        side = torch.zeros(g.V, dtype=torch.uint8, device=dev)
        with wbpr.Solver(0, max_wall_ms=120_000) as solver:
            solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)  # warm-up
            ms, scans = [], 0
            for _ in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1000.0)
                scans += st["arc_scans"]
        ms.sort()
        v = int(value.item())
        out[name] = {"graph": g.name, "V": g.V, "E": g.E, "ms_per_solve": round(ms[len(ms) // 2], 3),
                     "arc_scans_per_s": round(scans / (sum(ms) / 1e3), 1), "max_flow": v,
                     "equals_oracle": v == gold[name]["value"], "lds_resident": bool(st["lds_solved"]),
                     "generated_s": round(gen_s, 1)}
        log(f"[bench] {name}: {out[name]}")
        del rp, col, cap, flow, side
    return out


def layout_time(g, rp, col, cap, dev, layout, steps=3):
    """Median solve time of the headline graph in another residual layout."""
    import torch

    from paper_2404_00270_amd import wbpr

    value = torch.zeros(1, dtype=torch.int64, device=dev)
    flow = torch.zeros(max(g.E, 1), dtype=torch.int32, device=dev)
    side = torch.zeros(g.V, dtype=torch.uint8, device=dev)
    with wbpr.Solver(0, max_wall_ms=120_000, layout=layout) as solver:
        solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
        ms = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1000.0)
    ms.sort()
    return ms[len(ms) // 2], int(value.item())


def _stream_golden(n):
    path = os.path.join(ROOT, "tests", "golden", "batch_stream_values.txt")
    vals = {}
    if os.path.exists(path):
        with open(path) as f:
            for ln in f:
                if ln.startswith("#") or not ln.strip():
                    continue
                parts = ln.split()
                vals[int(parts[0])] = int(parts[3])
    return [vals.get(i) for i in range(n)]


def stream_leg(n, dev, rates, group=256, budget=1 << 30, slots=256, seed=5):
    """The batched and served stream: n instances solved one at a time, in
    device batches of `group`, through the server with all queued at once,
    and through the server with Poisson arrivals at each rate multiple of
    the one-at-a-time throughput."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    t0 = time.perf_counter()
    with ThreadPoolExecutor(16) as ex:  # the generator releases the GIL
        gs = list(ex.map(W.batch_instance, range(n)))
    gen_s = time.perf_counter() - t0
    Vs = [g.V for g in gs]
    Es = [g.E for g in gs]
    Vt, Et = sum(Vs), sum(Es)
    log(f"[bench] stream: {n} instances, V={Vt} E={Et}, generated in {gen_s:.1f}s")
    rp = torch.from_numpy(np.concatenate([g.row_ptr for g in gs]).astype(np.int64)).to(dev)
    col = torch.from_numpy(np.concatenate([g.col for g in gs]).astype(np.int32)).to(dev)
    cap = torch.from_numpy(np.concatenate([g.cap for g in gs]).astype(np.int32)).to(dev)
    vals = [torch.zeros(n, dtype=torch.int64, device=dev) for _ in range(2)]
    flows = [torch.zeros(max(Et, 1), dtype=torch.int32, device=dev) for _ in range(2)]
    sides = [torch.zeros(Vt, dtype=torch.uint8, device=dev) for _ in range(2)]
    ro = np.concatenate([[0], np.cumsum([v + 1 for v in Vs])])
    eo = np.concatenate([[0], np.cumsum(Es)])
    vo = np.concatenate([[0], np.cumsum(Vs)])
    torch.cuda.synchronize()
    out = {"instances": n, "V_total": Vt, "E_total": Et,
           "recipe": f"batch_instance(0..{n - 1}): V log-uniform [256, 65536], 8V distinct uniform arcs, caps "
                     "U[1,100], s = 0, t = V - 1; every route writes values, flows and cut sides"}
    with wbpr.Solver(0, max_wall_ms=300_000) as solver:
        def solve_one(i, k=0):
            g = gs[i]
            wbpr.wbpr_solve_device(solver.ctx, g.V, g.E, rp.data_ptr() + 8 * int(ro[i]),
                                   col.data_ptr() + 4 * int(eo[i]), cap.data_ptr() + 4 * int(eo[i]), g.s, g.t, 0,
                                   vals[k].data_ptr() + 8 * i, flows[k].data_ptr() + 4 * int(eo[i]),
                                   sides[k].data_ptr() + int(vo[i]))

        def solve_group(a, b):
            return wbpr.wbpr_solve_batch_device(
                solver.ctx, Vs[a:b], Es[a:b], [g.s for g in gs[a:b]], [g.t for g in gs[a:b]],
                rp.data_ptr() + 8 * int(ro[a]), col.data_ptr() + 4 * int(eo[a]), cap.data_ptr() + 4 * int(eo[a]), 0,
                vals[1].data_ptr() + 8 * a, flows[1].data_ptr() + 4 * int(eo[a]), sides[1].data_ptr() + int(vo[a]))

        # warm-up: the arena grows to the largest instance and the largest group once
        solve_one(int(np.argmax(Es)))
        big_group = max(range(0, n, group), key=lambda a: sum(Es[a:a + group]))
        solve_group(big_group, min(n, big_group + group))
        t0 = time.perf_counter()
        for i in range(n):
            solve_one(i)
        t_single = time.perf_counter() - t0
        t0 = time.perf_counter()
        for a in range(0, n, group):
            solve_group(a, min(n, a + group))
        t_batch = time.perf_counter() - t0
        same = bool(torch.equal(vals[0], vals[1]) and torch.equal(sides[0], sides[1]))
        alone_v = vals[0].cpu().numpy()
        alone_s = sides[0].cpu().numpy()
        gold = _stream_golden(n)
        out["one_at_a_time"] = {"solves_per_s": round(n / t_single, 1), "ms": round(t_single * 1e3, 1)}
        out["batched_groups"] = {"solves_per_s": round(n / t_batch, 1), "ms": round(t_batch * 1e3, 1),
                                 "group": group, "identical_to_one_at_a_time": same}
        out["values_equal_oracle"] = all(gv is not None and int(alone_v[i]) == gv for i, gv in enumerate(gold))
        log(f"[bench] stream one-at-a-time {out['one_at_a_time']} batched {out['batched_groups']}")
        r1 = n / t_single
        served = []
        for mult in [None] + list(rates):
            rate = None if mult is None else mult * r1
            leg = served_leg(solver, gs, rate, alone_v, alone_s, vo, budget, slots, seed)
            leg["rate_multiple_of_one_at_a_time"] = mult
            served.append(leg)
            log(f"[bench] served {'saturating' if mult is None else f'{mult}x'}: {leg}")
        out["served"] = served
    out["generated_s"] = round(gen_s, 1)
    return out


def served_leg(solver, gs, rate, alone_values, alone_sides, vo, budget=1 << 30, slots=256, seed=5):
    """Requests into the continuous-batching server: Poisson arrivals at `rate`
    per second, or all queued at once (rate None: the server's capacity)."""
    import numpy as np

    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(gs)) if rate else np.zeros(len(gs))
    tickets = [None] * len(gs)
    with wbpr.Server(solver, hbm_budget_bytes=budget, max_slots=slots) as srv:
        def producer():
            t_next = time.perf_counter()
            for i, g in enumerate(gs):
                t_next += gaps[i]
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(g)

        t0 = time.perf_counter()
        th = threading.Thread(target=producer)
        th.start()
        th.join()
        res = [srv.wait(tk, 300_000) for tk in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
    ok = all(r is not None and r.status == 0 for r in res)
    same = ok and all(int(r.value) == int(alone_values[i]) and
                      np.array_equal(r.side, alone_sides[vo[i]:vo[i + 1]]) for i, r in enumerate(res))
    return {
        "arrival_rate_per_s": round(rate, 1) if rate else "all queued at once",
        "solves_per_s": round(st["solves_per_s"], 1),
        "wall_solves_per_s": round(len(gs) / wall, 1),
        "p50_ms": round(st["p50_ms"], 2),
        "p99_ms": round(st["p99_ms"], 2),
        "max_ms": round(st["max_ms"], 2),
        "peak_resident": st["peak_resident"],
        "rounds": st["rounds"],
        "hbm_budget_bytes": budget,
        "identical_to_alone": bool(same),
    }


def ablation(workloads, dev, steps=2):
    """The paper's comparison (its Tables 1-2) on the synthetic stand-ins:
    thread-centric (one thread per active vertex) versus vertex-centric
    (tiles of lanes) on both residual layouts, BCSR and RCSR, each with the
    paper's full-scan active-vertex queue and with the incremental queue.
    Every variant must give the same value."""
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    # every variant runs the rounds of sweep launches (lds_max_v = -1) without
    # the gap heuristic (gap = -1): the comparison is between the paper's
    # sweep kernels, not the LDS-resident solve or the added heuristic
    variants = []
    for lay, ln in ((1, "BCSR"), (2, "RCSR")):
        variants += [
            (f"VC+{ln}, incremental queue", dict(layout=lay, lds_max_v=-1, gap=-1)),
            (f"VC+{ln}, full-scan queue", dict(layout=lay, avq_mode=1, lds_max_v=-1, gap=-1)),
            (f"TC+{ln}, full-scan queue", dict(layout=lay, lanes_per_vertex=1, avq_mode=1, lds_max_v=-1, gap=-1)),
            (f"TC+{ln}, incremental queue", dict(layout=lay, lanes_per_vertex=1, lds_max_v=-1, gap=-1)),
        ]
    out = []
    for name in workloads:
        g = W.WORKLOADS[name]()
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        cap = torch.from_numpy(g.cap).to(dev)
        value = torch.zeros(1, dtype=torch.int64, device=dev)
        flow = torch.zeros(max(g.E, 1), dtype=torch.int32, device=dev)
        side = torch.zeros(g.V, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        row = {"workload": g.name}
        values = set()
        for label, opts in variants:
            solver = wbpr.Solver(0, max_wall_ms=60_000, **opts)
            try:
                solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)  # warm-up
                t0 = time.perf_counter()
                for _ in range(steps):
                    solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
                torch.cuda.synchronize()
                row[label] = round((time.perf_counter() - t0) * 1000.0 / steps, 2)
                values.add(int(value.item()))
            except wbpr.WbprError as e:
                row[label] = f"not finished: {e}"
            finally:
                solver.close()
            log(f"[ablation] {g.name} {label}: {row[label]}")
        row["same_value"] = len(values) == 1
        for ln in ("BCSR", "RCSR"):  # the paper's speed-up column: TC time / VC time, same layout
            tc, vc = row.get(f"TC+{ln}, full-scan queue"), row.get(f"VC+{ln}, full-scan queue")
            if isinstance(tc, float) and isinstance(vc, float):
                row[f"speedup_vc_over_tc_{ln}"] = round(tc / vc, 2)
        out.append(row)
    return out


def wave_spread(tr):
    """Per-wave execution times normalised by the mean of their launch, over
    the waves that had work: (std-dev, p50, p90, p99, max, waves)."""
    import numpy as np

    busy = tr[tr[:, 4] > 0]
    keys = busy[:, 0] * 4 + busy[:, 1]
    order = np.argsort(keys, kind="stable")
    keys, t = keys[order], busy[order, 2].astype(np.float64)
    bounds = np.flatnonzero(np.diff(keys)) + 1
    norm = [x / x.mean() for x in np.split(t, bounds) if len(x) > 1 and x.mean() > 0]
    if not norm:
        return None
    v = np.concatenate(norm)
    q = np.percentile(v, [50, 90, 99])
    return dict(std=round(float(v.std()), 3), p50=round(float(q[0]), 3), p90=round(float(q[1]), 3),
                p99=round(float(q[2]), 3), max=round(float(v.max()), 2), waves=int(len(v)))


def wave_trace_study(workloads, dev):
    """The paper's workload analysis (section 5): every wave's execution time,
    normalised by its launch's mean, for the thread-centric and the
    vertex-centric kernel (both with the full-scan queue of Algorithm 2, as
    the paper's comparison), and for the default schedule."""
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    variants = [("TC, full-scan queue", dict(lanes_per_vertex=1, avq_mode=1)),
                ("VC, full-scan queue", dict(avq_mode=1)),
                ("VC, default schedule", {})]
    out = []
    for name in workloads:
        g = W.WORKLOADS[name]()
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        cap = torch.from_numpy(g.cap).to(dev)
        value = torch.zeros(1, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        row = {"workload": g.name}
        for label, opts in variants:
            with wbpr.Solver(0, max_wall_ms=60_000, wave_trace=1, **opts) as solver:
                solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value)  # warm-up (graph capture)
                st = solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value)
                tr = solver.wave_trace()
            row[label] = dict(spread=wave_spread(tr), records=int(len(tr)), ms=round(st["ms_total"], 2),
                              value=int(value.item()))
            log(f"[wave-trace] {g.name} {label}: {row[label]}")
        out.append(row)
    return out


def multi_terminal_study(workloads, pairs=20, seed=1, steps=2):
    """The paper's protocol for graphs without terminals (section 4): `pairs`
    source/sink pairs chosen by BFS among the vertices farthest apart, joined
    by a super-source and a super-sink; selection time and solve time."""
    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    out = []
    for name in workloads:
        g = W.WORKLOADS[name]()
        with wbpr.Solver(0, max_wall_ms=120_000) as solver:
            t0 = time.perf_counter()
            src, snk = solver.pick_terminals(g, pairs, seed)
            t1 = time.perf_counter()
            r = solver.solve_multi(g, src, snk)  # warm-up
            ms = []
            for _ in range(steps):
                r = solver.solve_multi(g, src, snk)
                ms.append(r.stats["ms_total"])
            ecc, _ = solver.bfs_farthest(g, src)
        row = {"workload": g.name, "pairs": int(len(src)), "ecc_min": int(ecc.min()), "ecc_max": int(ecc.max()),
               "select_ms": round((t1 - t0) * 1000.0, 1), "solve_ms": round(min(ms), 2), "value": r.value,
               "note": "solve_ms: GPU solve of the graph with super-source and super-sink (host arrays in, "
                       "PCIe included)"}
        log(f"[multi] {row}")
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel-steps", type=int, default=1, help="instrumented solves for the per-kernel roofline")
    ap.add_argument("--workload", default="rmat", choices=["plain", "bipartite", "rmat", "grid"])
    ap.add_argument("--layout", type=int, default=0, help="residual layout of the timed steps (1 BCSR, 2 RCSR)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream", type=int, default=4096, help="instances of the batched/served stream (0: skip)")
    ap.add_argument("--stream-rates", default="0.25,0.5,1,2",
                    help="served arrival rates, multiples of the one-at-a-time throughput")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--no-rcsr", action="store_true", help="skip the headline graph in the RCSR layout")
    ap.add_argument("--no-flows", action="store_true", help="value and cut only (skips the second phase)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--gr-every", type=int, default=0)
    ap.add_argument("--gr-permille", type=int, default=0)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--block-degree", type=int, default=0)
    ap.add_argument("--push-mode", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of this many MiB (HBM counter calibration)")
    ap.add_argument("--ablation", default="", metavar="W1,W2",
                    help="only run the thread-centric / vertex-centric comparison on these workloads")
    ap.add_argument("--wave-trace", default="", metavar="W1,W2",
                    help="only run the per-wave workload analysis on these workloads")
    ap.add_argument("--multi-terminal", default="", metavar="W1,W2",
                    help="only run the paper's 20-pair super-source/super-sink protocol on these workloads")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build measures a single MI355X.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.ablation:
        print(json.dumps({"ablation": ablation(args.ablation.split(","), dev)}), flush=True)
        return
    if args.wave_trace:
        print(json.dumps({"wave_trace": wave_trace_study(args.wave_trace.split(","), dev)}), flush=True)
        return
    if args.multi_terminal:
        print(json.dumps({"multi_terminal": multi_terminal_study(args.multi_terminal.split(","))}), flush=True)
        return
    if args.calibrate_copy > 0:
        # a plain copy reads and writes exactly n bytes each: the reference
        # for scaling FETCH_SIZE / WRITE_SIZE counters
        n = args.calibrate_copy << 20
        x = torch.ones(n // 4, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return
    t0 = time.perf_counter()
    g = W.WORKLOADS[args.workload]()
    log(f"[bench] generated {g.name}: V={g.V} E={g.E} in {time.perf_counter() - t0:.1f}s")

    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    cap = torch.from_numpy(g.cap).to(dev)
    value = torch.zeros(1, dtype=torch.int64, device=dev)
    flow = None if args.no_flows else torch.zeros(max(g.E, 1), dtype=torch.int32, device=dev)
    side = torch.zeros(g.V, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    opts = dict(lanes_per_vertex=args.lanes, gr_every_sweeps=args.gr_every, gr_work_permille=args.gr_permille,
                split_degree=args.split, block_degree=args.block_degree, push_mode=args.push_mode,
                grid_blocks=args.blocks, no_graph=int(args.no_graph), layout=args.layout, max_wall_ms=300_000)
    solver = wbpr.Solver(0, **opts)

    def step():
        return solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)

    for i in range(args.warmup):
        st = step()
        log(f"[bench] warmup {i}: {st['ms_total']:.1f} ms value={int(value.item())}")

    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, st in enumerate(stats):
        log(f"[bench] step {i}: total {st['ms_total']:.1f} ms (build {st['ms_build']:.1f}, solve {st['ms_phase1']:.1f}) "
            f"sweeps={st['sweeps']} gr={st['global_relabels']} scans={st['arc_scans']} pushes={st['pushes']} "
            f"relabels={st['relabels']} graph={st['use_graph']}")
    flow_value = int(value.item())
    ms_per_step = elapsed * 1000.0 / args.steps
    scans = sum(st["arc_scans"] for st in stats)
    arc_scans_per_s = scans / elapsed

    # instrumented solves: HIP events around every launch on the library's stream
    kstats = []
    if args.kernel_steps > 0:
        solver.set_options(**opts, time_kernels=1)
        for i in range(args.kernel_steps):
            kstats.append(step())
            log(f"[bench] instrumented {i}: total {kstats[-1]['ms_total']:.1f} ms kernel_ms={kstats[-1]['kernel_ms']} "
                f"build_ms={kstats[-1]['kernel_build_ms']:.2f}")
        solver.set_options(**opts)
        assert int(value.item()) == flow_value
    kernels = kernel_table(kstats) if kstats else None
    roofline, secondary = roofline_of(kstats, kernels) if kstats else (None, [])
    if args.workload == "rmat" and args.layout in (0, 1):
        # counter bytes per launch, as `achieved`: the family's and the
        # builder's per-solve counts spread over their launches per solve
        if roofline is not None:
            tr = measured_traffic("sweep", "rmat_s22")
            per_solve_launches = roofline["launches"] / len(kstats)
            roofline["traffic"] = round(tr / per_solve_launches, 1) if tr else None
        for sec in secondary:
            tr = measured_traffic("relabel" if sec["kernel"] == KERNELS[3] else "builder", "rmat_s22")
            sec["traffic"] = round(tr, 1) if tr else None
    solver.close()

    # the CPU oracle on the headline graph, in the background from here on
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle (FIFO push-relabel and Dinic) started on the headline graph")
        cpu = CpuBaseline(g).start()

    out = {
        "metric": "max-flow solve time & arc-scans/s (GB/s vs HBM peak); batched solves/s + p99",
        "value": arc_scans_per_s,
        "unit": "arc-scans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic",
        "config": {
            "workload": g.name,
            "V": g.V,
            "E": g.E,
            "M": stats[-1]["M"] if stats else None,
            "s": g.s,
            "t": g.t,
            "max_flow": flow_value,
            "flows": not args.no_flows,
            "layout": "RCSR" if stats and stats[-1]["layout"] == 2 else "BCSR",
            "lanes_per_vertex": stats[-1]["lanes_per_vertex"] if stats else None,
            "split_degree": stats[-1]["split_degree"] if stats else None,
            "block_degree": stats[-1]["block_degree"] if stats else None,
            "gr_every_sweeps": stats[-1]["gr_every_sweeps"] if stats else None,
            "sweeps_per_solve": stats[-1]["sweeps"] if stats else None,
            "global_relabels_per_solve": stats[-1]["global_relabels"] if stats else None,
            "ms_build": stats[-1]["ms_build"] if stats else None,
            "ms_solve": stats[-1]["ms_phase1"] if stats else None,
            "hipgraph": bool(stats[-1]["use_graph"]) if stats else None,
        },
        "roofline": roofline,
        "secondary": secondary,
        "kernels": kernels,
        "cpu_baseline": None,
        "workloads": None,
        "stream": None,
    }
    if args.layout in (0, 1) and not args.no_rcsr:
        rc_ms, rc_value = layout_time(g, rp, col, cap, dev, 2)
        out["rcsr_ms"] = round(rc_ms, 3)
        out["rcsr_same_value"] = rc_value == flow_value
        log(f"[bench] RCSR layout: {rc_ms:.1f} ms value={rc_value}")
    del rp, col, cap, flow, side
    torch.cuda.empty_cache()
    if not args.no_other_workloads:
        out["workloads"] = other_workloads([w for w in ("plain", "bipartite", "grid") if w != args.workload], dev)
    torch.cuda.empty_cache()
    if args.stream > 0:
        rates = [float(x) for x in args.stream_rates.split(",") if x]
        out["stream"] = stream_leg(args.stream, dev, rates)
    if cpu is not None:
        out["cpu_baseline"] = cpu.result(ms_per_step)
        if out["cpu_baseline"] is not None:
            out["cpu_baseline"]["same_value_as_gpu"] = all(v[1] == flow_value for v in cpu.res.values())
        log(f"[bench] cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
