"""Writes tests/golden/workload_values.json: oracle answers for the full-size
evaluation workloads.

Only the CPU oracle (oracle/) and the seeded input generators are called.
For each workload the file records the input hash (so a generator change is
caught), the maximum flow value on which both oracle solvers agree, the
capacity of the canonical cut (vertices that reach t in the residual graph of
the oracle's maximum flow) and a hash of that sink-side vector.

The batched stream (4,096 independent instances, `batch_instance(i)`) goes
to batch_stream_values.txt instead: one line per instance with V, E, the
value, the size of the canonical sink side and the first 16 hex digits of
its sha256, under a header holding the sha256 over every instance's input.

Usage:  python tests/golden/make_golden.py [plain bipartite rmat grid stream]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2404_00270_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "workload_values.json")
STREAM_OUT = os.path.join(HERE, "batch_stream_values.txt")
STREAM_N = 4096


def _stream_one(i):
    g = W.batch_instance(i)
    value, side, cutcap = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    if cutcap != value:
        raise RuntimeError(f"instance {i}: cut capacity {cutcap} != value {value}")
    return (i, g.V, g.E, value, int(side.sum()), hashlib.sha256(side.tobytes()).hexdigest()[:16],
            bytes.fromhex(g.sha256()))


def stream(n=STREAM_N):
    import multiprocessing as mp

    t0 = time.time()
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        rows = pool.map(_stream_one, range(n), chunksize=16)
    h = hashlib.sha256()
    for r in rows:
        h.update(r[6])
    with open(STREAM_OUT, "w") as f:
        f.write(f"# batched stream: {n} instances batch_instance(0..{n - 1}); oracle: dinic == fifo_pr, "
                f"certified by orc_check\n")
        f.write(f"# inputs_sha256 {h.hexdigest()}\n")
        f.write("# index V E value sink_side_size sink_side_sha256[:16]\n")
        for r in rows:
            f.write(" ".join(str(x) for x in r[:6]) + "\n")
    print(f"stream: {n} instances, sum V {sum(r[1] for r in rows)}, sum E {sum(r[2] for r in rows)}, "
          f"{time.time() - t0:.1f}s", flush=True)


def main(names):
    if "stream" in names:
        stream()
        names = [x for x in names if x != "stream"]
        if not names:
            return
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        t0 = time.time()
        g = W.WORKLOADS[name]()
        value, side, cutcap = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
        data[name] = {
            "graph": g.name,
            "graph_sha256": g.sha256(),
            "V": g.V,
            "E": g.E,
            "s": g.s,
            "t": g.t,
            "value": value,
            "cut_capacity": cutcap,
            "sink_side_size": int(side.sum()),
            "sink_side_sha256": hashlib.sha256(side.tobytes()).hexdigest(),
            "oracle": "dinic == fifo_pr, certified by orc_check",
        }
        print(name, data[name], f"{time.time() - t0:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["plain", "bipartite", "rmat", "grid"])
