"""GPU parity of the paper's subspace correction over the basis functions of
every level (Section "Multigrid Solution", ACSEG_FLAG_SSC) against the FP64
oracle.

The iteration changes only how a time step reaches its unique minimiser, so a
step is held to the gates of every other step (natural residual <= 1e-6,
max |u_gpu - u_oracle| <= 1e-4 from the oracle's state, labels), against the
oracle's truncated multigrid and against the oracle's own subspace correction.
The GPU visits a level's functions in four parity classes instead of row-major
order, which changes the iterates but not the fixed point.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import GATE_U, GPU_TOL, check_step, cuda, gpu_problem, host, label_gate, orc_params

pytestmark = pytest.mark.gpu


# (520, 40): six levels, so level 5's supports run in chunks over two launches
@pytest.mark.parametrize("W,H,N,levels,seed", [(96, 80, 4, 0, 1), (77, 130, 3, 3, 2), (64, 64, 2, 0, 3),
                                               (90, 70, 6, 2, 4), (45, 33, 8, 0, 5), (520, 40, 3, 0, 7)])
def test_ssc_step_parity_pixel_units(W, H, N, levels, seed):
    base = synth.pixel_twin(synth.VORONOI1024).scaled(W, H, N=N)
    img, u0, _ = base.make(seed)
    print(f"ssc step W={W} H={H} N={N} levels={levels} seed={seed}", flush=True)
    err, st, _, _ = check_step(base, img, u0, levels=levels, max_cycles=3000, flags=acseg.FLAG_SSC)
    assert st["cycles_max"] >= 1


def test_ssc_step_matches_oracle_subspace_correction():
    w = synth.pixel_twin(synth.VORONOI1024).scaled(60, 44, N=3)
    img, u0, _ = w.make(6)
    u0 = np.asarray(u0, np.float32)
    P = orc_params(w, tol=1e-11, levels=0, ssc=True)
    u_ref, c_ref, st_ref = orc.step(P, img, u0)
    assert st_ref["converged"] and st_ref["nonmonotone"] == 0
    p = gpu_problem(w, levels=0, max_cycles=3000, flags=acseg.FLAG_SSC)
    u_g, c_g, st = acseg.step(p, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK and st["final_residual"] <= GPU_TOL, st
    ug = host(u_g)
    assert np.abs(ug - u_ref).max() <= GATE_U
    assert np.abs(host(c_g) - c_ref).max() < 1e-5
    bad, total, raw = label_gate(ug, u_ref)
    assert bad <= 1e-3 * total, (bad, raw)


def test_ssc_and_truncated_multigrid_reach_the_same_step():
    w = synth.pixel_twin(synth.VORONOI1024, 256)
    img, u0, _ = w.make(5)
    p_tr = gpu_problem(w, levels=0, max_cycles=3000)
    p_ssc = gpu_problem(w, levels=0, max_cycles=3000, flags=acseg.FLAG_SSC)
    u_tr, _, st_tr = acseg.step(p_tr, cuda(img), cuda(u0))
    u_ssc, _, st_ssc = acseg.step(p_ssc, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    print("cycles: truncated", st_tr["cycles_max"], "subspace correction", st_ssc["cycles_max"], flush=True)
    assert st_tr["status"] == acseg.OK and st_ssc["status"] == acseg.OK, (st_tr, st_ssc)
    assert np.abs(host(u_tr) - host(u_ssc)).max() <= GATE_U


@pytest.mark.parametrize("fixed", [False, True])
def test_ssc_solve_every_step(fixed):
    w = synth.pixel_twin(synth.VORONOI1024, 64)
    img, u0, _ = w.make(8)
    steps = 4
    flags = acseg.FLAG_SSC | (acseg.FLAG_FIXED_CYCLES if fixed else 0)
    p = acseg.Problem.from_workload(w, levels=0, steps=steps, tol=GPU_TOL, max_cycles=600, flags=flags)
    u, c, st, traj = acseg.solve(p, cuda(img), cuda(u0), checkpoints=True)
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK, st
    tr = host(traj)
    P = orc_params(w, tol=1e-12, levels=0)
    c_prev = None
    for n in range(steps):
        un = tr[n]
        u_ref, c_ref, _ = orc.step(P, img, un, c_prev)
        assert np.abs(tr[n + 1] - u_ref).max() <= GATE_U, n
        c_prev = c_ref


def test_ssc_full_size_pixel_units():
    """The 1024 x 1024 pixel-unit image, 8 levels: the step converges, stays on
    the simplices, and agrees with the truncated multigrid step to the gate."""
    w = synth.pixel_twin(synth.VORONOI1024)
    img, u0, _ = w.make(0)
    print("ssc full size 1024x1024 N=4", flush=True)
    p_ssc = gpu_problem(w, levels=0, max_cycles=3000, flags=acseg.FLAG_SSC)
    p_tr = gpu_problem(w, levels=0, max_cycles=3000)
    u_ssc, _, st = acseg.step(p_ssc, cuda(img), cuda(u0))
    u_tr, _, st_tr = acseg.step(p_tr, cuda(img), cuda(u0))
    torch.cuda.synchronize()
    print("cycles: subspace correction", st["cycles_max"], "truncated", st_tr["cycles_max"], flush=True)
    assert st["status"] == acseg.OK and st["final_residual"] <= GPU_TOL, st
    us = host(u_ssc)
    assert us.min() >= 0 and np.abs(us.sum(0) - 1).max() < 1e-5
    assert np.abs(us - host(u_tr)).max() <= GATE_U
