"""Pins for the oracle's P1 assembly (Section "Finite Element Notation").

The oracle assembles the lumped mass <eta_p, 1> and stiffness <grad eta_p,
grad eta_q> triangle by triangle on the lattice split along (x,y)-(x+1,y+1).
Checked against: the domain area, the triangle count around each node,
exactness of P1 on linear functions, zero row sums, symmetry, the Kronecker
structure of the Neumann 5-point operator, and positive definiteness of
H = M/tau + eps A.
"""
import numpy as np
import pytest


def path_laplacian(n):
    L = np.zeros((n, n))
    for i in range(n - 1):
        L[i, i] += 1
        L[i + 1, i + 1] += 1
        L[i, i + 1] -= 1
        L[i + 1, i] -= 1
    return L


def halved_ends(n):
    d = np.ones(n)
    d[0] = d[-1] = 0.5
    return np.diag(d)


def dense_A(stencil):
    H, W = stencil.shape[:2]
    A = np.zeros((H * W, H * W))
    for y in range(H):
        for x in range(W):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    qx, qy = x + dx, y + dy
                    if 0 <= qx < W and 0 <= qy < H:
                        A[y * W + x, qy * W + qx] = stencil[y, x, dy + 1, dx + 1]
                    else:
                        assert stencil[y, x, dy + 1, dx + 1] == 0.0
    return A


def triangles_per_node(W, H):
    cnt = np.zeros((H, W))
    for cy in range(H - 1):
        for cx in range(W - 1):
            for tri in (((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)),
                        ((cx, cy), (cx + 1, cy + 1), (cx, cy + 1))):
                for (x, y) in tri:
                    cnt[y, x] += 1
    return cnt


@pytest.mark.parametrize("W,H,h", [(2, 2, 1.0), (5, 4, 0.25), (9, 7, 1 / 8), (16, 11, 1.0)])
def test_mass(orc, W, H, h):
    m, _ = orc.assemble(W, H, h)
    area = (W - 1) * (H - 1) * h * h
    assert abs(m.sum() - area) < 1e-12 * area
    # lumped P1 mass = (number of incident triangles) * (h^2/2) / 3
    assert np.allclose(m, triangles_per_node(W, H) * h * h / 6.0, rtol=0, atol=1e-15)
    if W > 2 and H > 2:
        assert m[0, 0] == pytest.approx(h * h / 3) and m[-1, -1] == pytest.approx(h * h / 3)
        assert m[0, -1] == pytest.approx(h * h / 6) and m[-1, 0] == pytest.approx(h * h / 6)


@pytest.mark.parametrize("W,H,h", [(5, 4, 0.25), (9, 7, 1 / 8), (6, 6, 1.0)])
def test_stiffness_kronecker_and_exactness(orc, W, H, h):
    m, s = orc.assemble(W, H, h)
    A = dense_A(s)
    # symmetric, zero row sums, 5-point Neumann structure (diagonal couplings vanish
    # on right triangles): A = D_y (x) L_x + L_y (x) D_x with halved boundary edges
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.allclose(A.sum(axis=1), 0, atol=1e-13)
    K = np.kron(halved_ends(H), path_laplacian(W)) + np.kron(path_laplacian(H), halved_ends(W))
    assert np.allclose(A, K, atol=1e-13)
    # P1 reproduces linear functions: u.A u = |grad u|^2 * area, lumped mass integrates them exactly
    X, Y = np.meshgrid(np.arange(W) * h, np.arange(H) * h)
    for a, b in [(1.0, 0.0), (0.0, 1.0), (0.7, -1.3)]:
        u = (a * X + b * Y).ravel()
        area = (W - 1) * (H - 1) * h * h
        assert u @ A @ u == pytest.approx((a * a + b * b) * area, rel=1e-12)
    area = (W - 1) * (H - 1) * h * h
    assert (m * X).sum() == pytest.approx(area * (W - 1) * h / 2, rel=1e-12)
    assert (m * Y).sum() == pytest.approx(area * (H - 1) * h / 2, rel=1e-12)


def test_step_operator_spd(orc):
    W, H, h = 6, 5, 1 / 5
    eps, tau = 2 * h, 4 * h * h
    P = orc.Params(H=H, W=W, C=1, N=1, h=h, eps=eps, lam=0.0, tau=tau)
    n = W * H
    Hm = np.stack([orc.apply_H(P, np.eye(n)[k].reshape(1, H, W)).ravel() for k in range(n)], 1)
    assert np.allclose(Hm, Hm.T, atol=1e-12)
    assert np.linalg.eigvalsh(Hm).min() > 0
    m, s = orc.assemble(W, H, h)
    assert np.allclose(Hm, np.diag(m.ravel()) / tau + eps * dense_A(s), atol=1e-12)


def test_auto_levels(orc):
    assert orc.auto_levels(64, 64) == 4
    assert orc.auto_levels(1024, 1024) == 8
    assert orc.auto_levels(4096, 4096) == 10
    assert orc.auto_levels(15, 15) == 1
