"""torch streams through the C ABI (wbpr_solve_device / wbpr_solve_batch_device).

The library shares torch's HIP runtime (one libamdhip64 in the process), so a
torch stream handle is a stream of the library's runtime: the solve must be
ordered after the work queued on it, and later work on it must see the
outputs.  The inputs are built on the stream by a chain of small kernels, so
a solve that did not wait for them would read unfinished capacities.
"""
import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_one_hip_runtime_in_process():
    import torch

    from paper_2404_00270_amd import wbpr

    wbpr.load_library()
    torch.zeros(1, device="cuda")
    libs = set()
    with open("/proc/self/maps") as f:
        for ln in f:
            if "libamdhip64" in ln:
                libs.add(ln.split()[-1])
    say(f"[streams] HIP runtimes mapped: {sorted(libs)}")
    assert len(libs) == 1, libs


def _staged_inputs(g, dev, steps=64):
    """CSR tensors whose capacities are produced on the current stream by
    `steps` kernels (cap = sum of steps slices of cap / steps, exact)."""
    import torch

    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    base = torch.from_numpy(g.cap.astype(np.int64)).to(dev)
    q, r = base // steps, base % steps
    cap = torch.zeros(g.E, dtype=torch.int64, device=dev)
    for _ in range(steps):
        cap += q
    cap += r
    return rp, col, cap.to(torch.int32)


@pytest.mark.parametrize("use_side", [True, False])
def test_solve_tensors_on_torch_stream(use_side):
    import torch

    from paper_2404_00270_amd import wbpr

    dev = torch.device("cuda:0")
    g = W.random_graph(6000, 48000, 1, 100, 41)
    want, want_side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
    stream = torch.cuda.Stream() if use_side else torch.cuda.current_stream(dev)
    say(f"[streams] side stream={use_side} handle={stream.cuda_stream}")
    with wbpr.Solver(0, lds_max_v=-1, max_wall_ms=120_000) as solver, torch.cuda.stream(stream):
        rp, col, cap = _staged_inputs(g, dev)
        value = torch.full((1,), -1, dtype=torch.int64, device=dev)
        flow = torch.full((g.E,), -1, dtype=torch.int32, device=dev)
        side = torch.full((g.V,), 7, dtype=torch.uint8, device=dev)
        solver.solve_tensors(g.V, rp, col, cap, g.s, g.t, value, flow, side)
        # consumers queued on the same stream see the results
        v2 = value * 1
        fsum = flow.to(torch.int64).sum()
        stream.synchronize()
    assert int(v2.item()) == want
    f = flow.cpu().numpy()
    chk = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, f)
    assert chk.feasible and chk.value == want and chk.cut_capacity == want
    assert int(fsum.item()) == int(f.astype(np.int64).sum())
    assert np.array_equal(side.cpu().numpy(), want_side)


def test_batch_device_on_torch_stream():
    import torch

    from paper_2404_00270_amd import wbpr

    dev = torch.device("cuda:0")
    gs = [W.random_graph(1500 + 500 * i, 8 * (1500 + 500 * i), 1, 100, 60 + i) for i in range(4)]
    refs = [oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t) for g in gs]
    stream = torch.cuda.Stream()
    rp_h = np.concatenate([g.row_ptr for g in gs])
    big = W.Graph(sum(g.V for g in gs), np.zeros(1, np.int64), np.concatenate([g.col for g in gs]),
                  np.concatenate([g.cap for g in gs]), 0, 1, "packed")
    with wbpr.Solver(0, max_wall_ms=120_000) as solver, torch.cuda.stream(stream):
        _, col, cap = _staged_inputs(big, dev)
        rp = torch.from_numpy(rp_h).to(dev)
        values = torch.full((len(gs),), -1, dtype=torch.int64, device=dev)
        sides = torch.zeros(sum(g.V for g in gs), dtype=torch.uint8, device=dev)
        wbpr.wbpr_solve_batch_device(solver.ctx, [g.V for g in gs], [g.E for g in gs], [g.s for g in gs],
                                     [g.t for g in gs], rp.data_ptr(), col.data_ptr(), cap.data_ptr(),
                                     stream.cuda_stream, values.data_ptr(), None, sides.data_ptr())
        vals = values * 1
        stream.synchronize()
    sd = sides.cpu().numpy()
    off = 0
    for i, (g, ref) in enumerate(zip(gs, refs)):
        assert int(vals[i].item()) == ref[0]
        assert np.array_equal(sd[off:off + g.V], ref[1])
        off += g.V
