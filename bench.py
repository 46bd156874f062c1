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
batches replayed as captured hipGraphs, no events).  "roofline" prices the
kernel with the largest share of GPU time by its algorithmic bytes per
launch over its average launch duration; durations come from HIP events
recorded on the library's stream around every launch of extra instrumented
solves of the same graph, run right after the timed region (events cannot
sit between the kernels of a captured batch).  "cpu_baseline" times the
CPU oracle (FIFO push-relabel) on a bounded sample: the same R-MAT recipe at
scale 20.  "batched" solves a sample of the batched stream (instances with
log-uniform V in [256, 65536], out-degree 8, capacities U[1,100]) once as a
single batch and once as one-at-a-time solves of the same instances, checks
the results are identical, and reports solves/s of both.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (bidirectional CSR, int32 residuals,
# int64 excesses, int32 heights):
#   sweep kernels  per arc-scan 12 B: entry {column, residual} 8 B + height of
#                  the column 4 B; per queued vertex 24 B: queue slot 4 + row
#                  bounds 8 + e(u) 8 + h(u) 4; per push 52 B: two residual
#                  atomics (2 x 8 B read+write), two excess atomics (2 x 16 B
#                  read+write), mate index 4 B; per relabel 4 B.
#   global relabel per top-down entry 12 B (entry 8 + head height 4); per
#                  bottom-up entry 9 B (entry 8 + visit code 1); per vertex
#                  and launch 17 B (height reset 4 + visit reset 1 + queue
#                  rebuild reads e 8 + h 4).
B_SCAN, B_QUEUED, B_PUSH, B_RELABEL = 12, 24, 52, 4
B_BFS_TD, B_BFS_BU, B_BFS_V = 12, 9, 17
KERNELS = ["k_sweep_tile", "k_sweep_tile<64> (medium rows)", "k_sweep_chunk (long-row chunks)", "k_global_relabel"]


def kernel_bytes(st, k):
    if k < 3:
        return (B_SCAN * st["kernel_arc_scans"][k] + B_QUEUED * st["kernel_queued"][k]
                + B_PUSH * st["kernel_pushes"][k] + B_RELABEL * st["kernel_relabels"][k])
    td = st["bfs_topdown_scans"]
    bu = st["bfs_scans"] - td
    return B_BFS_TD * td + B_BFS_BU * bu + B_BFS_V * st["V"] * st["kernel_launches"][3]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(scale: int = 20):
    import oracle
    from paper_2404_00270_amd import workloads as W

    g = W.rmat(scale, 16, 0.57, 0.19, 0.19, 1, 1000, 3)
    t0 = time.perf_counter()
    r = oracle.fifo_pr(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    dt = time.perf_counter() - t0
    return {
        "value": r.arc_scans / dt,
        "unit": "arc-scans/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle FIFO push-relabel (single thread) on the same R-MAT recipe at scale {scale} "
                  f"(V={g.V}, E={g.E}): {dt:.2f} s, {r.arc_scans} arc-scans, value {r.value}",
        "solve_s": dt,
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
    return kernels


def measured_traffic(kernel: str, workload: str):
    """Calibrated HBM bytes per launch from the committed rocprofv3 counter
    runs, or None when the kernel sources changed since they were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in rec["sources"])).hexdigest()
    if h != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"].get(kernel)


def roofline_of(stats, kernels):
    dom = max(range(4), key=lambda k: kernels[k]["ms"])
    if kernels[dom]["launches"] == 0 or kernels[dom]["ms"] <= 0:
        return None
    launches = kernels[dom]["launches"]
    per_launch_bytes = sum(kernel_bytes(st, dom) for st in stats) / launches
    avg_launch_s = kernels[dom]["ms"] / 1e3 / launches
    achieved = per_launch_bytes / avg_launch_s / 1e9
    return {
        "kernel": KERNELS[dom],
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": None,
        "launches": launches,
        "avg_launch_us": round(avg_launch_s * 1e6, 3),
        "algorithmic_bytes_per_launch": round(per_launch_bytes, 1),
    }


def batched_leg(solver, n, dev):
    """One batch of n stream instances vs n one-at-a-time solves (same outputs)."""
    import numpy as np
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    gs = [W.batch_instance(i) for i in range(n)]
    Vs = [g.V for g in gs]
    Es = [g.E for g in gs]
    rp = torch.from_numpy(np.concatenate([g.row_ptr for g in gs]).astype(np.int64)).to(dev)
    col = torch.from_numpy(np.concatenate([g.col for g in gs]).astype(np.int32)).to(dev)
    cap = torch.from_numpy(np.concatenate([g.cap for g in gs]).astype(np.int32)).to(dev)
    Vt, Et = sum(Vs), sum(Es)
    vals = [torch.zeros(n, dtype=torch.int64, device=dev) for _ in range(2)]
    flows = [torch.zeros(max(Et, 1), dtype=torch.int32, device=dev) for _ in range(2)]
    sides = [torch.zeros(Vt, dtype=torch.uint8, device=dev) for _ in range(2)]
    ro = np.concatenate([[0], np.cumsum([v + 1 for v in Vs])])
    eo = np.concatenate([[0], np.cumsum(Es)])
    vo = np.concatenate([[0], np.cumsum(Vs)])
    torch.cuda.synchronize()

    def one_at_a_time():
        for i, g in enumerate(gs):
            wbpr.wbpr_solve_device(solver.ctx, g.V, g.E, rp.data_ptr() + 8 * int(ro[i]),
                                   col.data_ptr() + 4 * int(eo[i]), cap.data_ptr() + 4 * int(eo[i]), g.s, g.t, 0,
                                   vals[0].data_ptr() + 8 * i, flows[0].data_ptr() + 4 * int(eo[i]),
                                   sides[0].data_ptr() + int(vo[i]))

    def batch():
        return wbpr.wbpr_solve_batch_device(solver.ctx, Vs, Es, [g.s for g in gs], [g.t for g in gs], rp.data_ptr(),
                                            col.data_ptr(), cap.data_ptr(), 0, vals[1].data_ptr(),
                                            flows[1].data_ptr(), sides[1].data_ptr())

    batch()  # warm: arena sized for the batch
    one_at_a_time()
    t0 = time.perf_counter()
    one_at_a_time()
    t_single = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = batch()
    t_batch = time.perf_counter() - t0
    same = bool(torch.equal(vals[0], vals[1]) and torch.equal(sides[0], sides[1]))
    served = served_leg(solver, gs, rate=2.0 * n / t_single, alone_values=vals[0].cpu().numpy(),
                        alone_sides=sides[0].cpu().numpy(), vo=vo)
    return {
        "instances": n,
        "V_total": Vt,
        "E_total": Et,
        "batched_solves_per_s": n / t_batch,
        "single_solves_per_s": n / t_single,
        "speedup": t_single / t_batch,
        "batched_ms": t_batch * 1e3,
        "single_ms": t_single * 1e3,
        "identical_values_and_cuts": same,
        "batched_rounds": st["global_relabels"],
        "batched_sweeps": st["sweeps"],
        "sample": f"batch_instance(0..{n - 1}): V log-uniform [256, 65536], out-degree 8, caps U[1,100]; "
                  "flows, cut sides and values written by both legs",
        "served": served,
    }


def served_leg(solver, gs, rate, alone_values, alone_sides, vo, budget=1 << 30, slots=256, seed=5):
    """Poisson arrivals at `rate` requests/s into the continuous-batching server."""
    import threading

    import numpy as np

    from paper_2404_00270_amd import wbpr

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(gs))
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
        "arrival_rate_per_s": rate,
        "solves_per_s": st["solves_per_s"],
        "wall_solves_per_s": len(gs) / wall,
        "p50_ms": st["p50_ms"],
        "p99_ms": st["p99_ms"],
        "max_ms": st["max_ms"],
        "peak_resident": st["peak_resident"],
        "rounds": st["rounds"],
        "admissions": st["admissions"],
        "hbm_budget_bytes": budget,
        "arena_bytes": st["arena_bytes"],
        "identical_to_alone": bool(same),
    }


def ablation(workloads, dev, steps=2):
    """The paper's thread-centric / vertex-centric comparison (its Tables 1-2)
    on the synthetic stand-ins, BCSR layout: one thread per active vertex
    versus tiles of lanes, each with the paper's full-scan active-vertex queue
    and with the incremental queue.  Every variant must give the same value."""
    import torch

    from paper_2404_00270_amd import workloads as W
    from paper_2404_00270_amd import wbpr

    # every variant runs the rounds of sweep launches (lds_max_v = -1) without
    # the gap heuristic (gap = -1): the comparison is between the paper's
    # sweep kernels, not the LDS-resident solve or the added heuristic
    variants = [
        ("VC, incremental queue (default)", dict(lds_max_v=-1, gap=-1)),
        ("VC, full-scan queue (Algorithm 2)", dict(avq_mode=1, lds_max_v=-1, gap=-1)),
        ("TC, full-scan queue (paper baseline)", dict(lanes_per_vertex=1, avq_mode=1, lds_max_v=-1, gap=-1)),
        ("TC, incremental queue", dict(lanes_per_vertex=1, lds_max_v=-1, gap=-1)),
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
        tc, vc = row.get("TC, full-scan queue (paper baseline)"), row.get("VC, full-scan queue (Algorithm 2)")
        if isinstance(tc, float) and isinstance(vc, float):
            row["paper_speedup_vc_over_tc"] = round(tc / vc, 2)
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="instances in the batched leg (0: skip)")
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
                grid_blocks=args.blocks, no_graph=int(args.no_graph), max_wall_ms=300_000)
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
            log(f"[bench] instrumented {i}: total {kstats[-1]['ms_total']:.1f} ms kernel_ms={kstats[-1]['kernel_ms']}")
        solver.set_options(**opts)
        assert int(value.item()) == flow_value
    kernels = kernel_table(kstats) if kstats else None
    roofline = roofline_of(kstats, kernels) if kstats else None
    if roofline is not None and args.workload == "rmat":
        roofline["traffic"] = measured_traffic(roofline["kernel"], "rmat_s22")

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
        "dtype": "int32",
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
        "kernels": kernels,
        "cpu_baseline": None,
        "batched": None,
    }
    if args.batch > 0:
        log(f"[bench] batched leg: {args.batch} stream instances")
        out["batched"] = batched_leg(solver, args.batch, dev)
        log(f"[bench] batched: {out['batched']}")
    if not args.no_cpu_baseline and args.workload == "rmat":
        log("[bench] timing the CPU oracle on the bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
