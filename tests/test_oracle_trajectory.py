"""Pins for the oracle's energy (eq. E) and its time trajectories.

* energy closed forms on one-hot labellings of noiseless piecewise-constant
  images and on the barycentric field;
* discrete energy decay: with the convex part implicit and the concave and
  fitting parts explicit, E(u^{n+1}) + |u^{n+1} - u^n|_M^2 / tau <= E(u^n);
* fixed points: a constant image with a barycentric or one-hot field;
* symmetries: transpose and 180-degree rotation of the lattice (both keep the
  diagonal split), phase permutation, channel permutation, adding a constant
  to the image, and scaling the image by s together with lambda by 1/s^2;
* post-processing (Section "Post-processing"): argmax labels, composite and
  rounded composite.
"""
import numpy as np
import pytest

from paper_0710_0736_amd import synth


def run(orc, w, img, u0, steps, **kw):
    P = orc.Params.from_workload(w, C=img.shape[0], **kw)
    return orc.solve(P, steps, img, u0)


def test_energy_closed_forms(orc):
    W, H, N = 12, 9, 3
    rng = np.random.default_rng(0)
    lab = np.zeros((H, W), np.int64)
    lab[:, 5:] = 1
    lab[6:, :] = 2
    col = rng.uniform(0, 1, (N, 3))
    img = col[lab].transpose(2, 0, 1)
    h = 0.1
    P = orc.Params(H=H, W=W, C=3, N=N, h=h, eps=0.3, lam=7.0, tau=0.01)
    E, parts = orc.energy(P, img, synth.one_hot(lab, N))
    # interface: eps * sum over lattice edges with differing labels of |A_pq|
    # (1 on interior edges, 1/2 on boundary edges)
    cut = 0.0
    for y in range(H):
        for x in range(W):
            if x + 1 < W and lab[y, x] != lab[y, x + 1]:
                cut += 0.5 if y in (0, H - 1) else 1.0
            if y + 1 < H and lab[y, x] != lab[y + 1, x]:
                cut += 0.5 if x in (0, W - 1) else 1.0
    assert parts[0] == pytest.approx(P.eps * cut, rel=1e-13)
    assert abs(parts[1]) < 1e-14 and abs(parts[2]) < 1e-12
    # barycentric field: no interface, concave part = area (1 - 1/N) / eps
    E, parts = orc.energy(P, img, np.full((N, H, W), 1.0 / N))
    area = (W - 1) * (H - 1) * h * h
    assert abs(parts[0]) < 1e-13
    assert parts[1] == pytest.approx(area * (1 - 1 / N) / P.eps, rel=1e-13)


@pytest.mark.parametrize("w", [synth.DISK64.scaled(32), synth.pixel_twin(synth.VORONOI1024, 32)],
                         ids=lambda w: w.name)
def test_energy_decay_and_simplex(orc, w):
    img, u0, _ = w.make(0)
    P = orc.Params.from_workload(w, tol=1e-11)
    uT, traj, ct, st = orc.solve(P, 8, img, u0)
    m, _ = orc.assemble(w.W, w.H, w.h)
    assert all(s["converged"] and s["nonmonotone"] == 0 for s in st)
    for n in range(traj.shape[0]):
        if n > 0:
            assert np.abs(traj[n].sum(0) - 1).max() < 1e-12
            assert traj[n].min() >= 0.0
    E = [orc.energy(P, img, traj[n])[0] for n in range(traj.shape[0])]
    for n in range(1, 8):
        dissip = (m[None] * (traj[n + 1] - traj[n]) ** 2).sum() / P.tau
        assert E[n + 1] + dissip <= E[n] + 1e-9 * abs(E[n])


@pytest.mark.parametrize("pixel", [False, True])
def test_constant_image_fixed_points(orc, pixel):
    W, H, N = 16, 12, 3
    h = 1.0 if pixel else 1 / 15
    img = np.ones((3, H, W)) * np.array([0.2, 0.5, 0.9])[:, None, None]
    P = orc.Params(H=H, W=W, C=3, N=N, h=h, eps=2 * h, lam=50.0, tau=4 * h * h, tol=1e-13)
    for u0 in (np.full((N, H, W), 1.0 / N), synth.one_hot(np.zeros((H, W), np.int64), N)):
        uT, traj, ct, st = orc.solve(P, 3, img, u0)
        assert np.abs(uT - u0).max() < 1e-12


def test_symmetries(orc):
    w = synth.pixel_twin(synth.VORONOI1024, 24)
    img, u0, _ = w.make(5)
    base, *_ = run(orc, w, img, u0, 4, tol=1e-12)
    t_img, t_u0 = img.transpose(0, 2, 1).copy(), u0.transpose(0, 2, 1).copy()
    tr, *_ = run(orc, w, t_img, t_u0, 4, tol=1e-12)
    assert np.abs(tr - base.transpose(0, 2, 1)).max() < 1e-8
    rot, *_ = run(orc, w, img[:, ::-1, ::-1].copy(), u0[:, ::-1, ::-1].copy(), 4, tol=1e-12)
    assert np.abs(rot - base[:, ::-1, ::-1]).max() < 1e-8
    perm = [2, 0, 3, 1]
    pp, *_ = run(orc, w, img, u0[perm].copy(), 4, tol=1e-12)
    assert np.abs(pp - base[perm]).max() < 1e-8
    cp, *_ = run(orc, w, img[[1, 2, 0]].copy(), u0, 4, tol=1e-12)
    assert np.abs(cp - base).max() < 1e-8
    # these two change the data by round-off only (c shifts / scales inexactly);
    # pixel-unit trajectories amplify such perturbations about fivefold per step
    sh, *_ = run(orc, w, img + 0.3, u0, 4, tol=1e-12)
    assert np.abs(sh - base).max() < 1e-6
    from dataclasses import replace
    w2 = replace(w, lam=w.lam / 4.0)
    sc, *_ = run(orc, w2, img * 2.0, u0, 4, tol=1e-12)
    assert np.abs(sc - base).max() < 1e-6


def test_labels_and_composites(orc):
    u = np.array([[[0.5, 0.2]], [[0.5, 0.3]], [[0.0, 0.5]]])  # N=3, H=1, W=2
    c = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, 2.0]])         # C=2
    lab, comp, rnd = orc.labels(u, c)
    assert lab.tolist() == [[0, 2]]  # tie -> lowest index
    assert np.allclose(comp[:, 0, 0], [0.5, 0.5]) and np.allclose(comp[:, 0, 1], [1.2, 1.3])
    assert np.allclose(rnd[:, 0, 0], c[0]) and np.allclose(rnd[:, 0, 1], c[2])
