"""GPU parity of the data pre-passes through the C ABI against the oracle.

* acseg_refine / acseg_sample: bit-exact (copies) against oracle/data.py, for
  several lattices, channel counts and refinement depths (0 and the maximum 8
  included), plus the documented argument errors;
* acseg_colour_space: within 1e-5 (L*a*b* / 100) of the FP64 oracle on random
  colours, the knots of both piecewise definitions, black, white and greys;
* a time step on refined data (a grayscale pixel image refined twice) against
  the oracle's step on the oracle's refinement, to the gates of the solver
  parity tests, and the pixel labels of a short solve.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from oracle import data as od
from paper_0710_0736_amd import acseg, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("W,H,P,r", [(2, 2, 1, 0), (5, 3, 2, 1), (33, 17, 3, 3), (130, 67, 4, 2),
                                     (7, 5, 1, 8), (300, 2, 2, 4)])
def test_refine_and_sample_match_oracle(W, H, P, r):
    rng = np.random.default_rng(W + H + r)
    a = rng.random((P, H, W)).astype(np.float32)
    f = acseg.refine(cuda(a), r)
    torch.cuda.synchronize()
    ref = od.refine(a.astype(np.float64), r)
    assert f.shape == ref.shape
    assert np.array_equal(host(f), ref)
    # sampling: the pixel nodes of the refined data, and of an arbitrary refined field
    assert np.array_equal(host(acseg.sample(f, W, H, r)), a.astype(np.float64))
    g = rng.random(ref.shape).astype(np.float32)
    assert np.array_equal(host(acseg.sample(cuda(g), W, H, r)), od.sample(g, r))


def test_refine_and_sample_reject_out_of_range():
    L = acseg.lib()
    x = torch.zeros(16, device=DEV)
    cx = acseg.ctx(0)
    p = x.data_ptr()
    for fn in (L.acseg_refine, L.acseg_sample):
        assert fn(cx, 1, 2, 2, 9, p, p, None) == acseg.ERR_INVALID_ARG      # r > 8
        assert fn(cx, 1, 1, 2, 0, p, p, None) == acseg.ERR_INVALID_ARG      # W < 2
        assert fn(cx, 0, 2, 2, 0, p, p, None) == acseg.ERR_INVALID_ARG      # no planes
        assert fn(cx, 1, 32769, 32769, 0, p, p, None) == acseg.ERR_INVALID_ARG  # > 2^30 nodes
        assert fn(cx, 1, 4097, 4097, 3, p, p, None) == acseg.ERR_INVALID_ARG    # refined > 2^30
        assert fn(cx, 1, 2, 2, 0, None, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_colour_space(cx, 2, 4, p, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_colour_space(cx, 0, -1, p, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_colour_space(cx, 0, 0, None, None, None) == acseg.OK


@pytest.mark.parametrize("kind", [acseg.LAB, acseg.AB])
def test_colour_space_matches_oracle(kind):
    rng = np.random.default_rng(7 + kind)
    rand = rng.random((3, 5000))
    knots = np.array([0.0, 0.04045, 0.04045 * (1 + 1e-6), 0.5, 1.0])
    grid = np.stack(np.meshgrid(knots, knots, knots, indexing="ij")).reshape(3, -1)
    # colours whose X/Xw, Y/Yw or Z/Zw sit near the CIE knot (6/29)^3 = 0.008856
    near = np.full((3, 64), 0.0) + np.linspace(0.08, 0.12, 64)
    rgb = np.concatenate([rand, grid, near], axis=1).astype(np.float32)
    got = host(acseg.colour_space(cuda(rgb).reshape(3, 1, -1), kind)).reshape(3 if kind == acseg.LAB else 2, -1)
    ref = od.srgb_to_lab(rgb.astype(np.float64), ab_only=(kind == acseg.AB))
    assert np.abs(got - ref).max() < 1e-5
    white = rand.shape[1] + grid.shape[1] - 1  # the last grid colour is (1, 1, 1)
    if kind == acseg.LAB:
        assert abs(got[0, white] - 1.0) < 1e-5 and np.abs(got[1:, white]).max() < 1e-5


def refined_problem(Wp, Hp, r, N, steps=1):
    Wf, Hf = acseg.refined_sides(Wp, Hp, r)
    h = 1.0 / (1 << r)  # pixel width 1
    kw = dict(H=Hf, W=Wf, C=1, N=N, h=h, eps=2 * h, lam=40.0, tau=(2 * h) ** 2)
    P = orc.Params(levels=0, tol=1e-12, **kw)
    p = acseg.Problem(steps=steps, levels=1, tol=1e-6, max_cycles=400, **kw)
    return P, p


def test_refined_step_and_pixel_labels_match_oracle():
    Wp = Hp = 24
    r, N = 2, 5
    img_p, _ = synth.concentric_circles(Wp, Hp, seed=3)
    img_p = img_p.astype(np.float32)
    P, p = refined_problem(Wp, Hp, r, N)
    If = acseg.refine(cuda(img_p), r)
    img_f = od.refine(img_p.astype(np.float64), r)
    assert np.array_equal(host(If), img_f)
    u0 = synth.random_simplex_field(N, p.H, p.W, seed=4).astype(np.float32)
    u_ref, c_ref, st_ref = orc.step(P, img_f, u0)
    assert st_ref["converged"]
    u_g, c_g, st = acseg.step(p, If, cuda(u0))
    torch.cuda.synchronize()
    assert st["final_residual"] <= 1e-6, st
    ug = host(u_g)
    assert np.abs(ug - u_ref).max() <= 1e-4
    assert np.abs(host(c_g) - c_ref).max() < 1e-5
    # three steps, then the labels at the pixels
    P3, p3 = refined_problem(Wp, Hp, r, N, steps=3)
    uT_ref = orc.solve(P3, 3, img_f, u0, keep_trajectory=False)[0]
    uT, _, st3, _ = acseg.solve(p3, If, cuda(u0))
    torch.cuda.synchronize()
    up_g = host(acseg.sample(uT, Wp, Hp, r))
    up_r = od.sample(uT_ref, r)
    s = np.sort(up_r, axis=0)
    decided = (s[-1] - s[-2]) > 1e-3
    assert ((up_g.argmax(0) != up_r.argmax(0)) & decided).sum() <= 1e-3 * decided.size + 0.5


@pytest.mark.parametrize("W,H,P", [(2, 2, 1), (5, 3, 2), (130, 67, 3), (257, 9, 1)])
def test_mass_average_matches_oracle(W, H, P):
    rng = np.random.default_rng(W * H + P)
    img = rng.random((P, H, W)).astype(np.float32)
    got = host(acseg.mass_average(cuda(img)))
    ref = od.mass_average(img.astype(np.float64), 1.0)
    assert np.abs(got - ref).max() < 1e-6


def test_mass_average_rejects_bad_sizes():
    L = acseg.lib()
    x = torch.zeros(16, device=DEV)
    cx, p = acseg.ctx(0), x.data_ptr()
    assert L.acseg_mass_average(cx, 1, 1, 4, p, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_mass_average(cx, 0, 2, 2, p, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_mass_average(cx, 1, 32769, 32769, p, p, None) == acseg.ERR_INVALID_ARG


def test_consistent_mass_step_matches_oracle():
    """A GPU step on the mass average against the oracle's consistent-mass step,
    assembled from its definition (means u_i.M I / u_i.M 1, gradient lambda M F_i)."""
    W, H, N, C, h = 61, 43, 3, 3, 1.0
    kw = dict(H=H, W=W, C=C, N=N, h=h, eps=2 * h, lam=40.0, tau=(2 * h) ** 2)
    P = orc.Params(levels=0, tol=1e-12, **kw)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=8, channels=C)
    img64 = img.astype(np.float64)
    un = synth.random_simplex_field(N, H, W, seed=9).astype(np.float32)
    un64 = un.astype(np.float64)
    M = od.mass_matrix(W, H, h)
    m = np.asarray(M.sum(axis=1)).ravel()
    MI = np.stack([M @ img64[k].ravel() for k in range(C)])
    c = np.array([[un64[i].ravel() @ MI[k] / (un64[i].ravel() @ m) for k in range(C)] for i in range(N)])
    a = 1.0 / P.tau + 2.0 / P.eps
    b = np.stack([(m * a * un64[i].ravel()
                   - P.lam * (M @ sum((img64[k] - c[i, k]) ** 2 for k in range(C)).ravel())).reshape(H, W)
                  for i in range(N)])
    u_ref, st_ref = orc.solve_qp(P, b, un64)
    assert st_ref["converged"]
    p = acseg.Problem(steps=1, levels=1, tol=1e-6, max_cycles=400, **kw)
    Ia = acseg.mass_average(cuda(img))
    u_g, c_g, st = acseg.step(p, Ia, cuda(un))
    torch.cuda.synchronize()
    assert st["final_residual"] <= 1e-6, st
    assert np.abs(host(c_g) - c).max() < 1e-5
    assert np.abs(host(u_g) - u_ref).max() <= 1e-4


@pytest.mark.parametrize("W,H,P", [(2, 2, 1), (5, 3, 2), (130, 67, 3), (257, 9, 1)])
def test_simplex_average_matches_oracle(W, H, P):
    rng = np.random.default_rng(W * H + P + 1)
    img = rng.random((P, H, W)).astype(np.float32)
    got = host(acseg.simplex_average(cuda(img)))
    ref = od.simplex_average(img.astype(np.float64), 1.0)
    assert np.abs(got - ref).max() < 1e-6


def test_simplex_average_rejects_bad_sizes():
    L = acseg.lib()
    x = torch.zeros(16, device=DEV)
    cx, p = acseg.ctx(0), x.data_ptr()
    assert L.acseg_simplex_average(cx, 1, 1, 4, p, p, None) == acseg.ERR_INVALID_ARG
    assert L.acseg_simplex_average(cx, 0, 2, 2, p, p, None) == acseg.ERR_INVALID_ARG


def test_simplex_projection_step_matches_oracle():
    """A GPU step on the by-simplex view against the oracle step assembled element
    by element (element values I_t, means int u_i I / int u_i, gradient
    sum_t (I_t - c_i)^2 |t| / 3), solved by the oracle's own QP solver."""
    W, H, N, C, h = 41, 33, 3, 3, 1.0
    kw = dict(H=H, W=W, C=C, N=N, h=h, eps=2 * h, lam=40.0, tau=(2 * h) ** 2)
    P = orc.Params(levels=0, tol=1e-12, **kw)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=10, channels=C)
    img64 = img.astype(np.float64)
    un = synth.random_simplex_field(N, H, W, seed=11).astype(np.float32)
    un64 = un.astype(np.float64)
    area = h * h / 2.0
    m = np.zeros((H, W))
    num = np.zeros((N, C))
    mass = np.zeros(N)
    tris = []
    for cy in range(H - 1):
        for cx in range(W - 1):
            for t in (((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)), ((cx, cy), (cx, cy + 1), (cx + 1, cy + 1))):
                It = sum(img64[:, y, x] for x, y in t) / 3.0
                tris.append((t, It))
                for x, y in t:
                    m[y, x] += area / 3.0
                for i in range(N):
                    num[i] += It * area * sum(un64[i, y, x] for x, y in t) / 3.0
    for i in range(N):
        mass[i] = (m * un64[i]).sum()
    c = num / mass[:, None]
    a = 1.0 / P.tau + 2.0 / P.eps
    b = np.stack([m * a * un64[i] for i in range(N)])
    for t, It in tris:
        for i in range(N):
            f = ((It - c[i]) ** 2).sum()
            for x, y in t:
                b[i, y, x] -= P.lam * area / 3.0 * f
    u_ref, st_ref = orc.solve_qp(P, b, un64)
    assert st_ref["converged"]
    p = acseg.Problem(steps=1, levels=1, tol=1e-6, max_cycles=400, **kw)
    Is = acseg.simplex_average(cuda(img))
    u_g, c_g, st = acseg.step(p, Is, cuda(un))
    torch.cuda.synchronize()
    assert st["final_residual"] <= 1e-6, st
    assert np.abs(host(c_g) - c).max() < 1e-5
    assert np.abs(host(u_g) - u_ref).max() <= 1e-4
