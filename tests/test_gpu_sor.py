"""GPU parity of the over-relaxed smoother (ACSEG_FLAG_SOR) against the FP64 oracle.

Over-relaxation changes only the path to a time step's unique minimiser, so its
steps meet the gates of every other step (natural residual <= 1e-6,
max |u_gpu - u_oracle| <= 1e-4 from the oracle's state, labels), in pixel units
(omega about 1.67) and at the unit scale (omega about 1).  In pixel units it
must also need fewer cycles than plain Gauss-Seidel.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import GATE_U, check_step, cuda, gpu_problem, host, orc_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,H,N,levels,seed", [(96, 80, 4, 1, 1), (77, 130, 3, 1, 2), (64, 64, 2, 1, 3),
                                               (90, 70, 6, 1, 4), (45, 33, 8, 1, 5), (120, 90, 4, 0, 6)])
def test_sor_step_parity_pixel_units(W, H, N, levels, seed):
    base = synth.pixel_twin(synth.VORONOI1024).scaled(W, H, N=N)
    img, u0, _ = base.make(seed)
    print(f"sor step W={W} H={H} N={N} levels={levels} seed={seed}", flush=True)
    check_step(base, img, u0, levels=levels, max_cycles=2000, flags=acseg.FLAG_SOR)


def test_sor_step_parity_unit_scale():
    w = synth.VORONOI1024.scaled(200, 150)
    img, u0, _ = w.make(2)
    check_step(w, img, u0, levels=1, max_cycles=200, flags=acseg.FLAG_SOR)


def test_sor_needs_fewer_cycles_in_pixel_units():
    w = synth.pixel_twin(synth.VORONOI1024, 256)
    img, u0, _ = w.make(5)
    p_gs = gpu_problem(w, levels=1, max_cycles=2000)
    p_sor = gpu_problem(w, levels=1, max_cycles=2000, flags=acseg.FLAG_SOR)
    u_gs, _, st_gs = acseg.step(p_gs, cuda(img), cuda(u0))
    u_sor, _, st_sor = acseg.step(p_sor, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    print("cycles: Gauss-Seidel", st_gs["cycles_max"], "over-relaxed", st_sor["cycles_max"], flush=True)
    assert st_gs["status"] == acseg.OK and st_sor["status"] == acseg.OK, (st_gs, st_sor)
    assert np.abs(host(u_gs) - host(u_sor)).max() <= GATE_U
    assert 2 * st_sor["cycles_max"] < st_gs["cycles_max"], (st_sor, st_gs)


@pytest.mark.parametrize("fixed", [False, True])
def test_sor_solve_every_step(fixed):
    w = synth.pixel_twin(synth.VORONOI1024, 64)
    img, u0, _ = w.make(8)
    steps = 4
    flags = acseg.FLAG_SOR | (acseg.FLAG_FIXED_CYCLES if fixed else 0)
    p = acseg.Problem.from_workload(w, levels=1, steps=steps, tol=1e-6, max_cycles=400, flags=flags)
    u, c, st, traj = acseg.solve(p, cuda(img), cuda(u0), checkpoints=True)
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK, st
    tr = host(traj)
    P = orc_params(w, tol=1e-12, levels=0)
    c_prev = None
    for n in range(steps):
        u_ref, c_ref, _ = orc.step(P, img, tr[n], c_prev)
        assert np.abs(tr[n + 1] - u_ref).max() <= GATE_U, n
        c_prev = c_ref


def test_batched_sor_equals_single_image_solves():
    """The batched kernel's over-relaxed variant gives each image exactly what a
    single-image solve gives it."""
    ws = [synth.pixel_twin(synth.VORONOI1024).scaled(96, 72), synth.pixel_twin(synth.VORONOI1024).scaled(64, 80, N=3)]
    probs = [acseg.Problem.from_workload(w, levels=1, steps=3, max_cycles=40, tol=1e-6,
                                         flags=acseg.FLAG_SOR | acseg.FLAG_FIXED_CYCLES) for w in ws]
    made = [w.make(11 + k) for k, w in enumerate(ws)]
    us = [cuda(m[1]) for m in made]
    _, cs, st = acseg.solve_batched(probs, [cuda(m[0]) for m in made], us)
    assert all(x["status"] == acseg.OK for x in st), st
    for p, m, u, c in zip(probs, made, us, cs):
        u1, c1, s1, _ = acseg.solve(p, cuda(m[0]), cuda(m[1]))
        torch.cuda.synchronize()
        assert s1["status"] == acseg.OK, s1
        assert torch.equal(u, u1) and torch.equal(c, c1)


def test_backward_through_an_over_relaxed_forward():
    """A solve with over-relaxed sweeps reaches the same steps, so its checkpoints
    give the oracle adjoint's gradients (the oracle runs on those checkpoints)."""
    from dataclasses import replace
    from test_gpu_adjoint import rel_err, setup
    w, p, img, u0, y = setup(True, 40, 32, 3, 3, 3, 1500)
    p = replace(p, flags=p.flags | acseg.FLAG_SOR)
    I = cuda(img)
    u, _, st, ck = acseg.solve(p, I, cuda(u0), checkpoints=True)
    assert st["status"] == acseg.OK, st
    gT = 2 * (u - cuda(y))
    gI, gu0, gp, gc, bst = acseg.backward(p, I, ck, gT)
    torch.cuda.synchronize()
    assert bst["status"] == acseg.OK, bst
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    Ibar, grads, cbar, ubar0 = orc.backward(P, 3, img, host(ck), host(gT))
    assert rel_err(host(gI), Ibar) <= 2e-3 and rel_err(host(gu0), ubar0) <= 2e-3
    g = gp.cpu().numpy()
    for k in range(3):
        assert abs(g[k] - grads[k]) <= 2e-3 * abs(grads[k]) + 1e-9, (k, g[k], grads[k])


def test_over_relaxed_fixed_schedule_solve_replays_equal_eager():
    w = synth.pixel_twin(synth.VORONOI1024, 96)
    p = acseg.Problem.from_workload(w, levels=1, steps=3, max_cycles=12,
                                    flags=acseg.FLAG_FIXED_CYCLES | acseg.FLAG_SOR)
    img, u0, _ = w.make(4)
    I, U0 = cuda(img), cuda(u0)
    u_ref, c_ref, st, _ = acseg.solve(p, I, U0.clone())
    assert st["status"] in (acseg.OK, acseg.WARN_NOT_CONVERGED), st
    u = U0.clone()
    acseg.solve(p, I, u, want_stats=False)  # warm-up (workspace, code objects)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        u.copy_(U0)
        _, c, _, _ = acseg.solve(p, I, u, want_stats=False)
    for k in range(3):
        u.fill_(0.25)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, u_ref) and torch.equal(c, c_ref), k
