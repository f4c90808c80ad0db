"""GPU gradients through a solve against the FP64 oracle's adjoint.

Both sides differentiate the same discrete trajectory: the oracle runs its
backward pass on the GPU's float32 checkpoints (so the free sets agree), and
the gradients are compared relative to their scale.  The oracle's adjoint is
pinned by finite differences in test_oracle_adjoint.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import GATE_U, cuda, host

pytestmark = pytest.mark.gpu


def setup(pixel, W, H, N, steps, seed, max_cycles):
    base = synth.pixel_twin(synth.VORONOI1024) if pixel else synth.VORONOI512
    w = base.scaled(W, H, N=N, steps=steps)
    img, u0, lab = w.make(seed)
    p = acseg.Problem.from_workload(w, C=3, levels=1, steps=steps, tol=1e-6, max_cycles=max_cycles)
    y = np.stack([(lab == i) for i in range(N)]).astype(np.float32)
    return w, p, img, u0, y


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("pixel,W,H,N,steps,seed,max_cycles", [
    (False, 96, 80, 4, 5, 1, 50),
    (False, 37, 53, 3, 3, 2, 50),
    (True, 40, 32, 3, 3, 3, 1500),
])
def test_backward_matches_oracle(pixel, W, H, N, steps, seed, max_cycles):
    w, p, img, u0, y = setup(pixel, W, H, N, steps, seed, max_cycles)
    I = cuda(img)
    u, _, st, ck = acseg.solve(p, I, cuda(u0), checkpoints=True)
    assert st["status"] == acseg.OK, st
    gT = 2 * (u - cuda(y))
    gI, gu0, gp, gc, bst = acseg.backward(p, I, ck, gT)
    torch.cuda.synchronize()
    assert bst["status"] == acseg.OK and bst["steps_done"] == steps, bst
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    Ibar, grads, cbar, ubar0 = orc.backward(P, steps, img, host(ck), host(gT))
    assert rel_err(host(gI), Ibar) <= 2e-3
    assert rel_err(host(gu0), ubar0) <= 2e-3
    assert rel_err(host(gc), cbar) <= 2e-3
    g = gp.cpu().numpy()
    for k in range(3):
        assert abs(g[k] - grads[k]) <= 2e-3 * abs(grads[k]) + 1e-9, (k, g[k], grads[k])


def test_segment_function_autograd():
    w, p, img, u0, y = setup(False, 64, 48, 3, 3, 4, 50)
    I = cuda(img).requires_grad_(True)
    U0 = cuda(u0).requires_grad_(True)
    lam = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(p.eps, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(p.tau, dtype=torch.float64, requires_grad=True)
    uT = acseg.SegmentFn.apply(I, U0, lam, eps, tau, p)
    loss = ((uT - cuda(y)) ** 2).sum()
    loss.backward()
    # the same gradients as a direct call
    u, _, _, ck = acseg.solve(p, cuda(img), cuda(u0), checkpoints=True)
    gI, gu0, gp, _, _ = acseg.backward(p, cuda(img), ck, 2 * (u - cuda(y)))
    torch.cuda.synchronize()
    assert torch.equal(uT.detach(), u)
    assert torch.allclose(I.grad, gI) and torch.allclose(U0.grad, gu0)
    assert torch.allclose(torch.stack([lam.grad, eps.grad, tau.grad]), gp.cpu())


@pytest.mark.parametrize("pixel", [False, True])
def test_fixed_means_forward_and_backward(pixel):
    w, p, img, u0, y = setup(pixel, 48, 40, 3, 3, 5, 1500 if pixel else 50)
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    c0, _ = orc.colour_means(P, img, u0)
    cf = (c0 + 0.05).astype(np.float32)
    I = cuda(img)
    u, c, st, ck = acseg.solve(p, I, cuda(u0), checkpoints=True, c_fixed=cuda(cf))
    torch.cuda.synchronize()
    assert st["status"] == acseg.OK, st
    assert np.array_equal(host(c), cf.astype(np.float64))  # an input, untouched
    ckh = host(ck)
    for n in range(p.steps):  # every step with the fixed means, from the GPU's own state
        u_ref, _, _ = orc.solve_fixed_c(P, 1, img, ckh[n], cf, keep_trajectory=False)
        assert np.abs(ckh[n + 1] - u_ref).max() <= GATE_U, n
    gT = 2 * (u - cuda(y))
    gI, gu0, gp, gc, bst = acseg.backward(p, I, ck, gT, c_fixed=cuda(cf))
    torch.cuda.synchronize()
    assert gc.shape == (3, 3) and bst["status"] == acseg.OK
    Ibar, grads, cbar, ubar0 = orc.backward_fixed_c(P, p.steps, img, ckh, cf, host(gT))
    assert rel_err(host(gI), Ibar) <= 2e-3
    assert rel_err(host(gu0), ubar0) <= 2e-3
    assert rel_err(host(gc), cbar) <= 2e-3
    g = gp.cpu().numpy()
    for k in range(3):
        assert abs(g[k] - grads[k]) <= 2e-3 * abs(grads[k]) + 1e-9, (k, g[k], grads[k])


def test_fixed_means_batched_equals_single():
    w, p, img, u0, y = setup(False, 64, 48, 3, 4, 6, 50)
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    cf = cuda(orc.colour_means(P, img, u0)[0] + 0.03)
    u_s, _, st_s, _ = acseg.solve(p, cuda(img), cuda(u0), c_fixed=cf)
    us, cs, sts = acseg.solve_batched([p, p], [cuda(img)] * 2, [cuda(u0), cuda(u0)], c_fixed=[cf, cf])
    torch.cuda.synchronize()
    assert torch.equal(us[0], u_s) and torch.equal(us[1], u_s)
    assert sts[0] == st_s


def test_differentiation_workload_at_full_size():
    """The differentiation workload itself (512^2 RGB, 4 Voronoi regions, N = 4,
    20 steps with every state checkpointed, loss = squared distance of u^20 to
    the one-hot ground truth): the forward against the oracle's trajectory, and
    the GPU gradients with respect to the image, u^0, lambda, eps, tau and every
    step's colour means against the FP64 oracle adjoint run on the GPU's
    checkpoints.  The oracle adjoint at this size is pinned by central
    differences in test_oracle_adjoint."""
    w = synth.VORONOI512
    img, u0, lab = w.make(0)
    y = np.stack([(lab == i) for i in range(w.N)]).astype(np.float32)
    p = acseg.Problem.from_workload(w, C=3, levels=1, tol=1e-6, max_cycles=50)
    I = cuda(img)
    u, _, st, ck = acseg.solve(p, I, cuda(u0), checkpoints=True)
    assert st["status"] == acseg.OK and st["steps_done"] == w.steps, st
    gT = 2 * (u - cuda(y))
    gI, gu0, gp, gc, bst = acseg.backward(p, I, ck, gT)
    torch.cuda.synchronize()
    assert bst["status"] == acseg.OK and bst["steps_done"] == w.steps, bst
    assert gc.shape == (w.steps, w.N, 3)
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    uT_ref, _, _, _ = orc.solve(P, w.steps, img, u0, keep_trajectory=False)
    assert np.abs(host(u) - uT_ref).max() <= GATE_U
    Ibar, grads, cbar, ubar0 = orc.backward(P, w.steps, img, host(ck), host(gT))
    assert rel_err(host(gI), Ibar) <= 2e-3
    assert rel_err(host(gu0), ubar0) <= 2e-3
    assert rel_err(host(gc), cbar) <= 2e-3
    g = gp.cpu().numpy()
    for k in range(3):
        assert abs(g[k] - grads[k]) <= 2e-3 * abs(grads[k]) + 1e-9, (k, g[k], grads[k])


def test_remembered_sweep_budget_rerun_and_reuse():
    """The context remembers the most adjoint sweeps a step of a problem took.
    A zero loss gradient converges at once, so a first call leaves a budget of
    two sweeps; a real gradient then needs more, runs again with host waits,
    and a third call, on the budget it left, must give the same result bit
    for bit (the sweeps after convergence do nothing)."""
    w, p, img, u0, y = setup(False, 72, 56, 3, 3, 5, 50)
    I = cuda(img)
    u, _, st, ck = acseg.solve(p, I, cuda(u0), checkpoints=True)
    assert st["status"] == acseg.OK, st
    _, _, _, _, b0 = acseg.backward(p, I, ck, torch.zeros_like(u))
    assert b0["status"] == acseg.OK and b0["cycles_max"] == 2, b0
    gT = 2 * (u - cuda(y))
    r1 = acseg.backward(p, I, ck, gT)
    r2 = acseg.backward(p, I, ck, gT)
    torch.cuda.synchronize()
    assert r1[4]["cycles_max"] > 2, r1[4]  # the remembered budget was too small
    assert r1[4] == r2[4], (r1[4], r2[4])
    for a, b in zip(r1[:4], r2[:4]):
        assert torch.equal(a, b)
    P = orc.Params.from_workload(w, C=3, tol=1e-12, levels=1)
    Ibar, grads, cbar, ubar0 = orc.backward(P, p.steps, img, host(ck), host(gT))
    assert rel_err(host(r2[0]), Ibar) <= 2e-3
    assert rel_err(host(r2[1]), ubar0) <= 2e-3
