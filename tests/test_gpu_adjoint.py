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
from test_gpu_parity import cuda, host

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
