"""Pins of the oracle's adjoint (the derivative of the time-step map).

The paper does not differentiate its scheme; the adjoint is derived from the
step's optimality conditions with the free sets held fixed.  It is pinned
against the forward oracle itself by finite differences (central, FP64, the
forward converged to 1e-13), against a dense pseudo-inverse on a tiny
lattice, and by the dot-product identity between the step's tangent map and
its adjoint.
"""
import numpy as np
import pytest

import oracle as orc
from paper_0710_0736_amd import synth


def small(pixel=True, W=10, H=8, N=3, lam=100.0, steps=3, seed=0):
    base = synth.pixel_twin(synth.VORONOI1024) if pixel else synth.VORONOI1024
    w = base.scaled(W, H, N=N, lam=lam, steps=steps)
    img, u0, lab = w.make(seed)
    P = orc.Params.from_workload(w, C=3, tol=1e-13, levels=1, max_cycles=200000)
    return w, P, img.astype(np.float64), u0.astype(np.float64), lab


def with_(P, **kw):
    d = dict(P.__dict__)
    d.update(kw)
    return type(P)(**d)


def test_adjoint_solve_is_the_derivative_of_the_qp():
    w, P, img, u0, _ = small()
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    u1, st = orc.solve_qp(P, b, u0)
    assert st["converged"]
    free = (u1 > 0).sum(0)
    assert (free == 1).any() and (free >= 2).any()  # both regimes present
    rng = np.random.default_rng(1)
    ubar = rng.standard_normal(u1.shape)
    db = rng.standard_normal(b.shape) * np.abs(b).mean()
    z = orc.adjoint_solve(P, u1, ubar)
    d = 1e-5  # inside one active set the map is affine: no truncation error
    up, _ = orc.solve_qp(P, b + d * db, u1)
    um, _ = orc.solve_qp(P, b - d * db, u1)
    assert ((up > 0) == (u1 > 0)).all() and ((um > 0) == (u1 > 0)).all()  # no active-set flip
    fd = ((up - um) * ubar).sum() / (2 * d)
    an = (z * db).sum()
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_adjoint_solve_matches_dense_pseudo_inverse():
    w, P, img, u0, _ = small(W=5, H=4, N=3)
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    u1, _ = orc.solve_qp(P, b, u0)
    n = P.W * P.H
    N = P.N
    # H as a dense matrix on one component, from unit vectors
    Hs = np.zeros((n, n))
    for q in range(n):
        e = np.zeros((N, P.H, P.W))
        e[0].flat[q] = 1.0
        Hs[:, q] = orc.apply_H(P, e)[0].ravel()
    Hf = np.kron(np.eye(N), Hs)  # component-major ordering, like the fields
    T = np.zeros((N * n, N * n))
    for p in range(n):
        idx = [i * n + p for i in range(N) if u1[i].flat[p] > 0]
        k = len(idx)
        if k >= 2:
            for a in idx:
                for bb in idx:
                    T[a, bb] = (1.0 if a == bb else 0.0) - 1.0 / k
    rng = np.random.default_rng(2)
    ubar = rng.standard_normal(N * n)
    z_ref = np.linalg.pinv(T @ Hf @ T) @ (T @ ubar)
    z = orc.adjoint_solve(P, u1, ubar.reshape(N, P.H, P.W)).ravel()
    assert np.abs(z - z_ref).max() <= 1e-9 * max(1.0, np.abs(z_ref).max())


def loss_and_target(w, P, img, u0, lab):
    y = np.stack([(lab == i).astype(np.float64) for i in range(P.N)])

    def L(Pp=P, I=img, u=u0):
        uT, _, _, _ = orc.solve(Pp, w.steps, I, u, keep_trajectory=False)
        return ((uT - y) ** 2).sum()

    return L, y


@pytest.mark.parametrize("pixel", [True, False])
def test_backward_matches_finite_differences(pixel):
    w, P, img, u0, lab = small(pixel=pixel)
    L, y = loss_and_target(w, P, img, u0, lab)
    uT, traj, _, _ = orc.solve(P, w.steps, img, u0)
    Ibar, grads, cbar, ubar0 = orc.backward(P, w.steps, img, traj, 2 * (uT - y))
    assert cbar.shape == (w.steps, P.N, P.C)
    rel = 1e-6

    def fd_param(name):
        v = getattr(P, name)
        d = rel * v
        return (L(Pp=with_(P, **{name: v + d})) - L(Pp=with_(P, **{name: v - d}))) / (2 * d)

    for k, name in enumerate(["lam", "eps", "tau"]):
        fd = fd_param(name)
        assert abs(fd - grads[k]) <= 1e-4 * max(abs(fd), 1e-8 * abs(L())), (name, fd, grads[k])
    rng = np.random.default_rng(3)
    V = rng.choice([-1.0, 1.0], size=img.shape)
    d = 1e-6
    fd = (L(I=img + d * V) - L(I=img - d * V)) / (2 * d)
    assert abs(fd - (Ibar * V).sum()) <= 1e-4 * max(abs(fd), 1e-6), (fd, (Ibar * V).sum())
    Vu = rng.standard_normal(u0.shape)
    fd = (L(u=u0 + d * Vu) - L(u=u0 - d * Vu)) / (2 * d)
    assert abs(fd - (ubar0 * Vu).sum()) <= 1e-4 * max(abs(fd), 1e-6), (fd, (ubar0 * Vu).sum())


def test_dot_product_identity_of_one_step():
    """<J v, w> = <v, J^T w> for the step map u^n -> u^{n+1} (J v by
    central differences of the forward step, J^T w by the adjoint)."""
    w, P, img, u0, _ = small(seed=4)
    u1, c, _ = orc.step(P, img, u0)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(u0.shape)
    wv = rng.standard_normal(u0.shape)
    d = 1e-7
    up, _, _ = orc.step(P, img, u0 + d * v)
    um, _, _ = orc.step(P, img, u0 - d * v)
    Jv = (up - um) / (2 * d)
    ubar_n, _, _, _ = orc.adjoint_step(P, img, u0, u1, wv)
    lhs, rhs_ = (Jv * wv).sum(), (v * ubar_n).sum()
    assert abs(lhs - rhs_) <= 1e-6 * max(1.0, abs(lhs)), (lhs, rhs_)


@pytest.mark.parametrize("pixel", [True, False])
def test_fixed_means_backward_matches_finite_differences(pixel):
    """With the colour means fixed (an input of the solve), the gradient with
    respect to them is a true input gradient: pinned by central differences of
    the forward oracle along every entry."""
    w, P, img, u0, lab = small(pixel=pixel, seed=6)
    c_fixed, _ = orc.colour_means(P, img, u0)
    c_fixed = c_fixed + 0.05  # away from the means of any state
    y = np.stack([(lab == i).astype(np.float64) for i in range(P.N)])

    def L(Pp=P, I=img, u=u0, c=c_fixed):
        uT, _, _ = orc.solve_fixed_c(Pp, w.steps, I, u, c, keep_trajectory=False)
        return ((uT - y) ** 2).sum()

    uT, traj, _ = orc.solve_fixed_c(P, w.steps, img, u0, c_fixed)
    Ibar, grads, cbar, ubar0 = orc.backward_fixed_c(P, w.steps, img, traj, c_fixed, 2 * (uT - y))
    d = 1e-6
    for i in range(P.N):
        for k in range(P.C):
            e = np.zeros_like(c_fixed)
            e[i, k] = d
            fd = (L(c=c_fixed + e) - L(c=c_fixed - e)) / (2 * d)
            assert abs(fd - cbar[i, k]) <= 1e-4 * max(abs(fd), 1e-6), (i, k, fd, cbar[i, k])
    for kk, name in enumerate(["lam", "eps", "tau"]):
        v = getattr(P, name)
        fd = (L(Pp=with_(P, **{name: v * (1 + d)})) - L(Pp=with_(P, **{name: v * (1 - d)}))) / (2 * d * v)
        assert abs(fd - grads[kk]) <= 1e-4 * max(abs(fd), 1e-8 * abs(L())), (name, fd, grads[kk])
    rng = np.random.default_rng(7)
    V = rng.choice([-1.0, 1.0], size=img.shape)
    fd = (L(I=img + d * V) - L(I=img - d * V)) / (2 * d)
    assert abs(fd - (Ibar * V).sum()) <= 1e-4 * max(abs(fd), 1e-6)
    Vu = rng.standard_normal(u0.shape)
    fd = (L(u=u0 + d * Vu) - L(u=u0 - d * Vu)) / (2 * d)
    assert abs(fd - (ubar0 * Vu).sum()) <= 1e-4 * max(abs(fd), 1e-6)


def test_differentiation_workload_finite_differences():
    """The differentiation workload at its own size (512^2 RGB, 4 Voronoi
    regions, sigma 0.1, N = 4, 20 steps, unit scale) with its finite-difference
    protocol: central differences of the FP64 forward with step 1e-3, absolute
    for lambda and for the image along a seeded Rademacher direction (every
    pixel-channel moves by 1e-3), relative for eps and tau.  The free sets of
    the +step and -step trajectories are compared component by component
    over all steps; a flip puts a kink between them, so the count is reported
    and the agreement is required where there is none."""
    w = synth.VORONOI512
    img, u0, lab = w.make(0)
    img, u0 = img.astype(np.float64), u0.astype(np.float64)
    P = orc.Params.from_workload(w, C=3, tol=1e-13, levels=1, max_cycles=200000)
    y = np.stack([(lab == i).astype(np.float64) for i in range(P.N)])
    uT, traj, _, _ = orc.solve(P, w.steps, img, u0)
    Ibar, grads, _, _ = orc.backward(P, w.steps, img, traj, 2 * (uT - y))

    def run(Pp=P, I=img):
        u, tr, _, _ = orc.solve(Pp, w.steps, I, u0)
        return ((u - y) ** 2).sum(), tr[1:] > 0

    def central(plus, minus, d):
        (Lp, fp), (Lm, fm) = plus, minus
        return (Lp - Lm) / (2 * d), int((fp != fm).sum())

    report = {}
    for k, (name, rel) in enumerate([("lam", False), ("eps", True), ("tau", True)]):
        v = getattr(P, name)
        d = 1e-3 * (v if rel else 1.0)
        fd, flips = central(run(Pp=with_(P, **{name: v + d})), run(Pp=with_(P, **{name: v - d})), d)
        report[name] = (fd, grads[k], flips)
    V = synth.rademacher(img.shape, seed=0).astype(np.float64)
    fd, flips = central(run(I=img + 1e-3 * V), run(I=img - 1e-3 * V), 1e-3)
    report["image"] = (fd, (Ibar * V).sum(), flips)
    print("finite differences (fd, adjoint, active-set flips):", report)
    for name, (fd, an, flips) in report.items():
        if flips == 0:
            assert abs(fd - an) <= 1e-3 * abs(fd), (name, fd, an)
    assert sum(r[2] for r in report.values()) == 0, report
