"""Solves captured in a HIP graph (through torch.cuda.graph).

With ACSEG_FLAG_FIXED_CYCLES, or ACSEG_FLAG_NO_HOST_WAIT (every cycle enqueued,
converged ones exiting on the device), and no statistics, acseg_solve enqueues
kernels and device copies only (control blocks are cleared by a kernel, never
by a memset), so a caller can capture a whole solve and replay it.  Each
replay, with eager work and synchronisations between replays, must reproduce
the eager solve bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("levels,early_exit", [(1, False), (0, False), (1, True), (0, True)])
def test_fixed_schedule_solve_replays_equal_eager(levels, early_exit):
    # early_exit: an adaptive schedule with every cycle enqueued (NO_HOST_WAIT); the
    # cycles after a step converges exit on the device, inside the graph too
    sched = acseg.FLAG_NO_HOST_WAIT if early_exit else acseg.FLAG_FIXED_CYCLES
    if levels == 1:
        w = synth.VORONOI1024.scaled(160, 120)
        p = acseg.Problem.from_workload(w, levels=1, steps=4, max_cycles=6 if early_exit else 2, flags=sched)
    else:
        w = synth.pixel_twin(synth.VORONOI1024, 96)
        p = acseg.Problem.from_workload(w, levels=0, steps=3, max_cycles=20, flags=sched)
    img, u0, _ = w.make(2)
    I, U0 = cuda(img), cuda(u0)
    u_ref, c_ref, st, _ = acseg.solve(p, I, U0.clone())
    assert st["status"] == acseg.OK, st

    u = torch.empty_like(U0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream before capture
        u.copy_(U0)
        acseg.solve(p, I, u, want_stats=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        u.copy_(U0)
        _, c, _, _ = acseg.solve(p, I, u, want_stats=False)
    for k in range(3):
        u.fill_(0.25)  # eager work between replays
        c.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, u_ref), k
        assert torch.equal(c, c_ref), k


def test_batched_solve_with_reused_tables_replays_equal_eager():
    """acseg_solve_batched with FLAG_REUSE_TABLES (tables left by an eager call with
    the same arguments) captured with labels and replayed three times, with eager
    work between replays: every replay equals the eager batched solve."""
    ws = [synth.VORONOI1024.scaled(160, 120), synth.VORONOI1024.scaled(96, 130, N=3),
          synth.VORONOI1024.scaled(200, 64)]
    probs = [acseg.Problem.from_workload(w, levels=1, steps=5, max_cycles=2, flags=acseg.FLAG_FIXED_CYCLES)
             for w in ws]
    made = [w.make(3 + k) for k, w in enumerate(ws)]
    imgs = [cuda(m[0]) for m in made]
    u0s = [cuda(m[1]) for m in made]
    us = [x.clone() for x in u0s]
    cs = [torch.empty((p.N, p.C), dtype=torch.float32, device="cuda") for p in probs]
    _, _, st = acseg.solve_batched(probs, imgs, us, cs=cs)
    assert all(x["status"] == acseg.OK for x in st), st
    u_ref = [x.clone() for x in us]
    c_ref = [x.clone() for x in cs]
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for b in range(len(us)):
            us[b].copy_(u0s[b])
        acseg.solve_batched(probs, imgs, us, want_stats=False, cs=cs, reuse_tables=True)
        labs = [acseg.labels(p, u, c)[0] for p, u, c in zip(probs, us, cs)]
    lab_ref = [acseg.labels(p, u, c)[0].clone() for p, u, c in zip(probs, u_ref, c_ref)]
    for k in range(3):
        for u, c in zip(us, cs):
            u.fill_(0.25)  # eager work between replays
            c.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b in range(len(us)):
            assert torch.equal(us[b], u_ref[b]), (k, b)
            assert torch.equal(cs[b], c_ref[b]), (k, b)
            assert torch.equal(labs[b], lab_ref[b]), (k, b)


def test_reuse_tables_refuses_other_arguments():
    """FLAG_REUSE_TABLES with arguments whose tables differ from the last upload is
    refused on the host, before anything is enqueued."""
    w = synth.VORONOI1024.scaled(96, 64)
    probs = [acseg.Problem.from_workload(w, levels=1, steps=2, max_cycles=1, flags=acseg.FLAG_FIXED_CYCLES)] * 2
    img, u0, _ = w.make(1)
    imgs = [cuda(img), cuda(img)]
    us = [cuda(u0), cuda(u0)]
    acseg.solve_batched(probs, imgs, us, want_stats=False)
    torch.cuda.synchronize()
    other = [cuda(u0), cuda(u0)]  # new output arrays: the uploaded tables point elsewhere
    with pytest.raises(acseg.AcsegError) as e:
        acseg.solve_batched(probs, imgs, other, want_stats=False, reuse_tables=True)
    assert e.value.code == acseg.ERR_INVALID_ARG
    # the same arguments are accepted (and give the same result as an upload)
    for x in us:
        x.copy_(cuda(u0))
    acseg.solve_batched(probs, imgs, us, want_stats=False, reuse_tables=True)
    ref = [cuda(u0), cuda(u0)]
    acseg.solve_batched(probs, imgs, ref, want_stats=False)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(us, ref))
