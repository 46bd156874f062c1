"""Writes tests/golden/workload_values.json: oracle answers for the full-size
evaluation workloads.

Only the CPU oracle (oracle/) and the seeded input generators are called.
For each workload the file records the input hash (so a generator change is
caught), the maximum flow value on which both oracle solvers agree, the
capacity of the canonical cut (vertices that reach t in the residual graph of
the oracle's maximum flow) and a hash of that sink-side vector.

Usage:  python tests/golden/make_golden.py [plain bipartite rmat grid]
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


def main(names):
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
