"""The device entry points inside a captured HIP graph.

The library allocates nothing and never synchronises on the device path, so a
fused step can be captured once (torch.cuda.graph records the launch on the
capture stream that the binding passes down) and replayed.  Each replay is
checked bit for bit against an eager launch on the same buffers, with eager
work between replays that rewrites the inputs and poisons the outputs, so a
replay that reused stale data or skipped a launch would show.
"""
import numpy as np
import pytest
import torch

import oracle
from _helpers import H, host_case, log

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def pw():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2010_01545_amd import pwadvect
    return pwadvect


@pytest.mark.parametrize("kernel", ["march", "direct"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fused_step_replays_in_a_graph(pw, dtype, kernel):
    log("graph %s %s" % (dtype, kernel))
    fields, lams, coef = host_case(37, 29, 64, 91, lam_seed=92)
    tzc1, tzc2, tcx, tcy = coef
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    st = [pw.pad_periodic(torch.from_numpy(a).to(DEV, dtype), H) for a in fields]
    sl = [pw.pad_periodic(torch.from_numpy(a).to(DEV, dtype), H) for a in lams]
    outs = [torch.zeros_like(st[0]) for _ in range(6)]
    prev = pw.set_kernel(kernel)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm-up launch off the default stream, as torch asks
            pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, H, out=outs)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, H, out=outs)
        for r in range(3):
            # eager work between replays: new inputs, poisoned outputs
            for q, t in enumerate(st):
                t.mul_(1.0 + 0.25 * r).add_(0.5 * q)
            for t in outs:
                t.fill_(float("nan"))
            ref = [o.clone() for o in pw.fwd_adj(*st, *sl, t1, t2, tcx, tcy, H)]
            for t in outs:
                t.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            for q, (g, e) in enumerate(zip(outs, ref)):
                gi, ei = oracle.interior(g.cpu().numpy(), H), oracle.interior(e.cpu().numpy(), H)
                assert np.array_equal(gi, ei), "replay %d output %d" % (r, q)
    finally:
        pw.set_kernel(prev)


@pytest.mark.parametrize("copy_out", ["auto", "runtime", "kernel", "direct"])
def test_static_offload_replays_in_a_graph(pw, copy_out):
    """The allocation-free offload (pw_advect_fwd_host_static) with pinned
    host fields, captured once and replayed: each replay matches an eager
    call bit for bit, with the host inputs rewritten and the host outputs
    poisoned between replays.  A captured call records and queries no timing
    events (the automatic copy-out mode uses what it measured before)."""
    log("graph offload %s" % copy_out)
    fields, _, coef = host_case(13, 11, 64, 93)
    tzc1, tzc2, tcx, tcy = coef
    t1, t2 = torch.from_numpy(tzc1).to(DEV), torch.from_numpy(tzc2).to(DEV)
    st = [oracle.pad_periodic(a, H) for a in fields]
    host_in = [torch.from_numpy(a).pin_memory() for a in st]
    outs = [torch.full(host_in[0].shape, float("nan"), dtype=torch.float64, pin_memory=True) for _ in range(3)]
    chunk = 4
    with pw.tuning(copy_out=copy_out):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm-up calls off the default stream (and timed, for "auto")
            for _ in range(3):
                pw.fwd_host_static(*host_in, t1, t2, tcx, tcy, H, *outs, chunk)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            pw.fwd_host_static(*host_in, t1, t2, tcx, tcy, H, *outs, chunk)
        torch.cuda.synchronize()
        for r in range(3):
            for q, t in enumerate(host_in):     # new host inputs (halos stay periodic: a scaled copy)
                t.copy_(torch.from_numpy(st[q] * (1.0 + 0.25 * r)))
            ref = [torch.full(o.shape, float("nan"), dtype=o.dtype, pin_memory=True) for o in outs]
            pw.fwd_host_static(*host_in, t1, t2, tcx, tcy, H, *ref, chunk)
            torch.cuda.synchronize()
            for t in outs:
                t.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            for q, (g, e) in enumerate(zip(outs, ref)):
                assert np.array_equal(oracle.interior(g.numpy(), H), oracle.interior(e.numpy(), H)), \
                    "replay %d output %d" % (r, q)
