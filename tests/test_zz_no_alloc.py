"""The allocation-free entry point (wbpr_solve_device_noalloc) against the
ordinary device entry point (wbpr_solve_device), both through the C ABI on
the same device-resident inputs: two calls in a row, the second on a smaller
graph (the static scratch array keeps the first call's contents and must be
cleared), in both residual layouts.  Values and canonical cut sides must be
identical, and both flows must pass the oracle's certificate (several
maximum flows are correct, so per-arc flows are compared by the
certificate, not bit for bit).  A graph too large for the array is refused
with WBPR_ETOOBIG, and the call made no device allocation: torch's and the
HIP runtime's view of free device memory do not shrink across it."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2404_00270_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _dev(g, torch, dev):
    return (torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), torch.from_numpy(g.cap).to(dev))


def _solve(fn, ctx, g, arrays, torch, dev):
    rp, col, cap = arrays
    value = torch.full((1,), -1, dtype=torch.int64, device=dev)
    flow = torch.full((max(g.E, 1),), -7, dtype=torch.int32, device=dev)
    side = torch.full((g.V,), 9, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = fn(ctx, g.V, g.E, rp.data_ptr(), col.data_ptr(), cap.data_ptr(), g.s, g.t, stream, value.data_ptr(),
            flow.data_ptr(), side.data_ptr())
    torch.cuda.synchronize()
    return int(value.item()), flow.cpu().numpy()[: g.E], side.cpu().numpy(), st


def _certify(g, value, flow):
    c = oracle.check(g.V, g.row_ptr, g.col, g.cap, g.s, g.t, flow)
    assert c.feasible, (g.name, c.code, c.bad)
    assert c.value == value and c.cut_capacity == value, g.name


def _free_bytes(torch):
    free, _ = torch.cuda.mem_get_info(0)
    return free


@pytest.mark.parametrize("layout", [1, 2])
def test_noalloc_equals_device_entry_point(layout):
    import torch

    from paper_2404_00270_amd import wbpr

    dev = torch.device("cuda:0")
    graphs = [W.random_graph(20000, 160000, 1, 100, 11), W.config_plain()]  # second call smaller
    inputs = [_dev(g, torch, dev) for g in graphs]
    with wbpr.Solver(0, layout=layout, max_wall_ms=60_000) as solver:
        for g, arrays in zip(graphs, inputs):
            say(f"[noalloc] layout={layout} {g.name} V={g.V} E={g.E}")
            want = _solve(wbpr.wbpr_solve_device, solver.ctx, g, arrays, torch, dev)
            got = _solve(wbpr.wbpr_solve_device_noalloc, solver.ctx, g, arrays, torch, dev)
            ref_value, ref_side, _ = oracle.reference(g.V, g.row_ptr, g.col, g.cap, g.s, g.t)
            assert got[0] == want[0] == ref_value, (g.name, got[0], want[0], ref_value)
            assert np.array_equal(got[2], want[2]) and np.array_equal(got[2], ref_side), g.name
            _certify(g, got[0], got[1])
            _certify(g, want[0], want[1])
            assert got[3]["use_graph"] == 0


def test_noalloc_allocates_nothing_and_refuses_too_large():
    import torch

    from paper_2404_00270_amd import wbpr

    dev = torch.device("cuda:0")
    g = W.random_graph(5000, 40000, 1, 100, 12)
    arrays = _dev(g, torch, dev)
    with wbpr.Solver(0, max_wall_ms=60_000) as solver:
        first = _solve(wbpr.wbpr_solve_device_noalloc, solver.ctx, g, arrays, torch, dev)  # loads the array
        torch.cuda.synchronize()
        before = _free_bytes(torch)
        for _ in range(3):
            again = _solve(wbpr.wbpr_solve_device_noalloc, solver.ctx, g, arrays, torch, dev)
            assert again[0] == first[0] and np.array_equal(again[2], first[2])
        assert _free_bytes(torch) >= before, "the allocation-free entry point allocated device memory"
        big = W.random_graph(1_000_000, 4_000_000, 1, 100, 13)
        say(f"[noalloc] too large: V={big.V} E={big.E}")
        big_arrays = _dev(big, torch, dev)
        with pytest.raises(wbpr.WbprError) as ei:
            _solve(wbpr.wbpr_solve_device_noalloc, solver.ctx, big, big_arrays, torch, dev)
        assert ei.value.code == wbpr.WBPR_ETOOBIG
        assert "allocation-free" in str(ei.value)
        # the context still works after the refusal
        after = _solve(wbpr.wbpr_solve_device_noalloc, solver.ctx, g, arrays, torch, dev)
        assert after[0] == first[0] and np.array_equal(after[2], first[2])
