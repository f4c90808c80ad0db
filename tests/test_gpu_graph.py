"""A fixed-schedule solve captured in a HIP graph (through torch.cuda.graph).

With ACSEG_FLAG_FIXED_CYCLES and no statistics, acseg_solve enqueues kernels
and device copies only (control blocks are cleared by a kernel, never by a
memset), so a caller can capture a whole solve and replay it.  Each replay,
with eager work and synchronisations between replays, must reproduce the
eager solve bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("levels", [1, 0])
def test_fixed_schedule_solve_replays_equal_eager(levels):
    if levels == 1:
        w = synth.VORONOI1024.scaled(160, 120)
        p = acseg.Problem.from_workload(w, levels=1, steps=4, max_cycles=2, flags=acseg.FLAG_FIXED_CYCLES)
    else:
        w = synth.pixel_twin(synth.VORONOI1024, 96)
        p = acseg.Problem.from_workload(w, levels=0, steps=3, max_cycles=20, flags=acseg.FLAG_FIXED_CYCLES)
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
