"""The streamed cycle (ACSEG_FLAG_STREAM: two sweeps, the residual and the
colour-mean partials in one launch down columns of the lattice) against the
FP64 oracle, against the tiled cycle, and batched against one image.

The streamed launch computes the same two global red-black sweeps as the
tiled one (every node update has the same operands); only the order of the
colour-mean partial sums differs, so one fixed cycle from the same state must
agree with the tiled launch to FP32 rounding, and a solve must hold the
oracle's per-step gates.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import GATE_U, GPU_TOL, check_step, cuda, gpu_problem, host, orc_params

pytestmark = pytest.mark.gpu

STREAM = acseg.FLAG_STREAM


@pytest.mark.parametrize("shape,N,C,pixel", [((65, 37), 3, 1, True), ((2, 2), 2, 3, True), ((3, 130), 4, 2, False),
                                             ((129, 66), 8, 4, True), ((70, 33), 5, 3, False),
                                             ((200, 150), 3, 3, True), ((160, 300), 6, 2, False),
                                             ((140, 90), 7, 1, True), ((54, 16), 4, 3, True),
                                             ((300, 280), 4, 3, False)])
def test_streamed_step_parity(shape, N, C, pixel):
    W, H = shape
    w = synth.Workload("ragged", W, H, N, "voronoi", 0.1, 40.0, 1, 0, 1e-6, pixel_units=pixel)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=7, channels=C)
    u0 = synth.random_simplex_field(N, H, W, seed=7)
    check_step(w, img, u0, C=C, flags=STREAM, max_cycles=600)


def test_streamed_full_size_headline_step():
    w = synth.VORONOI1024
    img, u0, _ = w.make(0)
    err, st, _, _ = check_step(w, img, u0, oracle_tol=1e-11, max_cycles=50, flags=STREAM)
    assert st["cycles_max"] <= 10


@pytest.mark.parametrize("w", [synth.VORONOI1024.scaled(300, 200), synth.pixel_twin(synth.VORONOI1024, 150),
                               synth.VORONOI4096.scaled(257, 129)], ids=lambda w: f"{w.name}_{w.W}x{w.H}")
def test_one_streamed_cycle_equals_one_tiled_cycle(w):
    """From the same state, one fixed cycle: the streamed and tiled launches
    make the same two global red-black sweeps."""
    img, u0, _ = w.make(3)
    p = gpu_problem(w, max_cycles=1, flags=acseg.FLAG_FIXED_CYCLES)
    ps = gpu_problem(w, max_cycles=1, flags=acseg.FLAG_FIXED_CYCLES | STREAM)
    u_t, c_t, st_t = acseg.step(p, cuda(img), cuda(u0))
    u_s, c_s, st_s = acseg.step(ps, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert np.abs(host(u_s) - host(u_t)).max() <= 2e-6
    assert torch.equal(c_s, c_t)  # the means of u^n: same reduction
    assert st_s["final_residual"] == pytest.approx(st_t["final_residual"], rel=1e-3, abs=1e-7)


@pytest.mark.parametrize("fixed", [False, True])
def test_every_step_of_a_streamed_solve(fixed):
    w = synth.pixel_twin(synth.VORONOI1024, 96)
    img, u0, _ = w.make(4)
    steps = 4
    flags = STREAM | (acseg.FLAG_FIXED_CYCLES if fixed else 0)
    p = gpu_problem(w, steps=steps, flags=flags, max_cycles=120 if fixed else 400)
    u, c, st, ck = acseg.solve(p, cuda(img), cuda(u0), checkpoints=True)
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK, st
    ck = host(ck)
    P = orc_params(w, tol=1e-12, levels=0)
    c_prev = None
    for n in range(steps):
        u_ref, c_used, _ = orc.step(P, img, ck[n], c_prev)
        assert np.abs(ck[n + 1] - u_ref).max() <= GATE_U, n
        c_prev = c_used


def test_streamed_trajectory_unit_scale():
    w = synth.VORONOI1024.scaled(256, 192, steps=10)
    img, u0, _ = w.make(5)
    P = orc_params(w, tol=1e-12, levels=0)
    _, traj, _, _ = orc.solve(P, w.steps, img, u0)
    p = gpu_problem(w, steps=w.steps, flags=STREAM)
    u, c, st, ck = acseg.solve(p, cuda(img), cuda(u0), checkpoints=True)
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK and st["max_residual"] <= GPU_TOL, st
    assert np.abs(host(ck) - traj).max() <= GATE_U


def test_batched_streamed_equals_single():
    specs = [(300, 200, 4, 3, 1), (97, 130, 3, 3, 2), (64, 64, 2, 1, 3), (180, 90, 5, 3, 4), (120, 260, 6, 3, 5)]
    problems, images, u0s = [], [], []
    for (W, H, N, C, seed) in specs:
        w = synth.VORONOI1024.scaled(W, H, N=N)
        img, u0, _ = w.make(seed)
        if C == 1:
            img = img.mean(axis=0, keepdims=True)
        problems.append(acseg.Problem.from_workload(w, C=C, levels=1, steps=5, tol=1e-6, max_cycles=20,
                                                    flags=STREAM))
        images.append(cuda(img))
        u0s.append(cuda(u0))
    singles = [acseg.solve(p, im, u0.clone())[:3] for p, im, u0 in zip(problems, images, u0s)]
    us, cs, sts = acseg.solve_batched(problems, images, [u.clone() for u in u0s])
    torch.cuda.synchronize()
    for b, (u, c, st) in enumerate(singles):
        assert torch.equal(us[b], u) and torch.equal(cs[b], c), b
        assert sts[b] == st and st["status"] == acseg.OK, (b, st)


def test_streamed_fixed_schedule_graph_replays():
    w = synth.VORONOI1024.scaled(200, 160, steps=4)
    img, u0, _ = w.make(6)
    p = gpu_problem(w, steps=4, max_cycles=1, flags=STREAM | acseg.FLAG_FIXED_CYCLES)
    I, U0 = cuda(img), cuda(u0)
    u = U0.clone()
    acseg.solve(p, I, u, want_stats=False, c_out=False)
    ref = u.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        u.copy_(U0)
        acseg.solve(p, I, u, want_stats=False, c_out=False)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ref)
        u.zero_()
        torch.cuda.synchronize()
