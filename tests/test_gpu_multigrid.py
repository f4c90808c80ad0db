"""GPU parity of the truncated multigrid correction (Section "Multigrid
Solution") against the FP64 oracle.

The multigrid only changes how fast a time step reaches its unique minimiser,
so a multigrid step is held to the same gates as a Gauss-Seidel step (natural
residual <= 1e-6, max |u_gpu - u_oracle| <= 1e-4 from the oracle's state), and
must need fewer cycles than Gauss-Seidel alone where Gauss-Seidel is slow
(pixel units).  The transfer operators are compared element by element with
the oracle's.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import GATE_U, GPU_TOL, check_step, cuda, gpu_problem, host, orc_params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Wf,Hf", [(2, 2), (3, 5), (9, 7), (10, 12), (33, 16), (64, 64), (129, 70)])
def test_transfer_matches_oracle(Wf, Hf):
    rng = np.random.default_rng(Wf * 1000 + Hf)
    Wc, Hc = (Wf + 1) // 2, (Hf + 1) // 2
    vc = rng.standard_normal((3, Hc, Wc)).astype(np.float32)
    vf = rng.standard_normal((3, Hf, Wf)).astype(np.float32)
    pg = host(acseg.prolong(cuda(vc), Wf, Hf))
    rg = host(acseg.restrict(cuda(vf)))
    torch.cuda.synchronize()
    pr = orc.prolong(vc.astype(np.float64), Wf, Hf)
    rr = orc.restrict(vf.astype(np.float64))
    assert np.abs(pg - pr).max() <= 1e-6 * max(1.0, np.abs(pr).max())
    assert np.abs(rg - rr).max() <= 4e-6 * max(1.0, np.abs(rr).max())
    # the two are transposes of each other on the GPU too: <P a, b> = <a, P^T b>
    lhs = float((pg.astype(np.float64) * vf).sum())
    rhs_ = float((vc.astype(np.float64) * rg).sum())
    assert abs(lhs - rhs_) <= 1e-4 * max(1.0, abs(lhs))


@pytest.mark.parametrize("W,H,N,seed", [(96, 80, 4, 1), (37, 53, 3, 2), (150, 150, 2, 3), (64, 128, 6, 4)])
def test_multigrid_step_parity_pixel_units(W, H, N, seed):
    base = synth.pixel_twin(synth.VORONOI1024).scaled(W, H, N=N)
    img, u0, _ = base.make(seed)
    err, st, _, _ = check_step(base, img, u0, levels=0, max_cycles=200)
    assert st["cycles_max"] >= 1


def test_multigrid_cuts_cycles_in_pixel_units():
    w = synth.pixel_twin(synth.VORONOI1024, 256)
    img, u0, _ = w.make(5)
    p_gs = gpu_problem(w, levels=1, max_cycles=2000)
    p_mg = gpu_problem(w, levels=0, max_cycles=2000)
    u_gs, _, st_gs = acseg.step(p_gs, cuda(img), cuda(u0))
    u_mg, _, st_mg = acseg.step(p_mg, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert st_gs["status"] == acseg.OK and st_mg["status"] == acseg.OK, (st_gs, st_mg)
    # same minimiser; a V(1,1) cycle costs about 3 sweeps, Gauss-Seidel 2 per cycle
    assert np.abs(host(u_gs) - host(u_mg)).max() <= GATE_U
    assert 3 * st_mg["cycles_max"] < 2 * st_gs["cycles_max"], (st_mg, st_gs)


def test_multigrid_full_size_unit_scale():
    """The headline image with its 8-level hierarchy: converges to the same
    step as Gauss-Seidel alone."""
    w = synth.VORONOI1024
    img, u0, _ = w.make(0)
    p_gs = gpu_problem(w, levels=1, max_cycles=50)
    p_mg = gpu_problem(w, levels=8, max_cycles=50)
    u_gs, _, st_gs = acseg.step(p_gs, cuda(img), cuda(u0))
    u_mg, _, st_mg = acseg.step(p_mg, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert st_mg["status"] == acseg.OK and st_mg["final_residual"] <= GPU_TOL, st_mg
    assert np.abs(host(u_gs) - host(u_mg)).max() <= 1e-5


@pytest.mark.parametrize("fixed", [False, True])
def test_every_step_of_a_multigrid_solve(fixed):
    w = synth.pixel_twin(synth.VORONOI1024, 72)
    img, u0, _ = w.make(7)
    steps = 4
    flags = acseg.FLAG_FIXED_CYCLES if fixed else 0
    p = gpu_problem(w, steps=steps, levels=0, flags=flags, max_cycles=40 if fixed else 200)
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


def test_multigrid_two_levels_and_odd_sizes():
    """Hierarchies that end on a large coarsest level (no LDS tail) and on
    odd sides."""
    w = synth.pixel_twin(synth.VORONOI1024).scaled(201, 131, N=3)
    img, u0, _ = w.make(9)
    for levels in (2, 3):
        check_step(w, img, u0, levels=levels, max_cycles=400)


@pytest.mark.parametrize("flags", [0, acseg.FLAG_SSC, acseg.FLAG_SOR], ids=["truncated", "ssc", "sor"])
def test_cycles_never_raise_the_step_objective(flags):
    """Every cycle (smoothing sweeps and the coarse correction) is a descent step
    of the step's strictly convex objective J: J after k + 1 fixed cycles is at
    most J after k (evaluated by the oracle in FP64 on the GPU's iterates, with
    a slack for their FP32 rounding), and it decreases overall."""
    w = synth.pixel_twin(synth.VORONOI1024).scaled(96, 80, N=4)
    img, u0, _ = w.make(12)
    u0 = np.asarray(u0, np.float32)
    P = orc_params(w, levels=0)
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    Js = []
    for k in range(1, 9):
        p = gpu_problem(w, levels=0, max_cycles=k, flags=acseg.FLAG_FIXED_CYCLES | flags)
        u_g, _, st = acseg.step(p, cuda(img), cuda(u0))
        torch.cuda.synchronize()
        ug = host(u_g).astype(np.float64)
        ug /= ug.sum(0, keepdims=True)  # onto the simplices in FP64 (FP32 sums miss 1 by rounding)
        Js.append(orc.objective(P, b, ug))
    slack = 1e-6 * abs(Js[0])
    assert all(Js[k + 1] <= Js[k] + slack for k in range(len(Js) - 1)), Js
    assert Js[-1] < Js[0]


@pytest.mark.parametrize("seed", [3, 4])
def test_stopped_step_equals_fixed_schedule_and_reports_its_residual(seed):
    """With V(1,1) every cycle closes with one launch of two sweeps (its
    post-smoothing and the next cycle's pre-smoothing), and the next cycle's
    defect pass tests convergence.  A step that stops after c cycles has then
    run exactly the launches of a fixed schedule of c cycles, so both return
    the same iterate bit for bit, and the residual the step reports is that
    iterate's natural residual (evaluated by the oracle in FP64)."""
    w = synth.pixel_twin(synth.VORONOI1024).scaled(160, 120, N=4)
    img, u0, _ = w.make(seed)
    u0 = np.asarray(u0, np.float32)
    p_ad = gpu_problem(w, levels=0, max_cycles=60)
    u_a, _, st_a = acseg.step(p_ad, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert st_a["status"] == acseg.OK and 1 <= st_a["cycles_max"] < 60, st_a
    p_fx = gpu_problem(w, levels=0, max_cycles=st_a["cycles_max"], flags=acseg.FLAG_FIXED_CYCLES)
    u_f, _, st_f = acseg.step(p_fx, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert torch.equal(u_a, u_f)
    assert st_f["final_residual"] == st_a["final_residual"], (st_a, st_f)
    P = orc_params(w, levels=0)
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    r = orc.residual(P, b, host(u_a).astype(np.float64))
    assert abs(r - st_a["final_residual"]) <= 2e-7 and r <= GPU_TOL + 2e-7, (r, st_a)


@pytest.mark.parametrize("nu_pre,nu_post", [(2, 1), (1, 2)])
def test_multigrid_step_parity_other_smoothing_counts(nu_pre, nu_post):
    """Cycles other than V(1,1) keep a pre-smoothing and a post-smoothing launch
    per cycle (the pre-smoothing launch makes the convergence test): the step
    still reaches the oracle's step."""
    w = synth.pixel_twin(synth.VORONOI1024).scaled(120, 96, N=4)
    img, u0, _ = w.make(15)
    check_step(w, img, u0, levels=0, max_cycles=400, nu_pre=nu_pre, nu_post=nu_post)
