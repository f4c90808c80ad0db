"""Pin of the oracle's step objective J(u) = sum_i [u_i.H u_i / 2 - b_i.u_i].

J judges every monotonicity check (the oracle's own count of coarse
corrections that raise it, and the GPU descent tests), so it is checked here
against a version written independently of the oracle's assembly:
  * the lumped mass of a node is h^2/6 times the number of lattice triangles
    that touch it (every cell split along its (x,y)-(x+1,y+1) diagonal);
  * u.A u is written as a sum over edges, sum_e w_e (u_p - u_q)^2, with the
    P1 cotangent weights w_e = (cot a + cot b) / 2 over the angles opposite
    the edge: 1/2 per right-isosceles triangle on a lattice edge, 0 on the
    diagonals (whose opposite angles are right angles);
  * H = M/tau + eps A (Section "Discretisation and Numerical Solution", with
    the stiffness entering positively).
Arbitrary fields (not on the simplex) and right-hand sides are used, so a
dropped factor, a wrong sign or a swapped operand in the oracle shows.
"""
import numpy as np
import pytest


def triangles_touching(W, H):
    """Number of lattice triangles incident to each node, [H][W]."""
    cnt = np.zeros((H, W))
    for cy in range(H - 1):
        for cx in range(W - 1):
            for tri in (((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)),
                        ((cx, cy), (cx + 1, cy + 1), (cx, cy + 1))):
                for (x, y) in tri:
                    cnt[y, x] += 1
    return cnt


def edge_energy(v):
    """v.A v for one field v [H][W] as a sum over lattice edges: an edge in
    the interior borders two triangles (weight 1/2 + 1/2), an edge on the
    boundary one (weight 1/2); diagonal edges carry no weight."""
    H, W = v.shape
    e = 0.0
    for y in range(H):
        for x in range(W):
            if x + 1 < W:
                w = 0.5 if y in (0, H - 1) else 1.0
                e += w * (v[y, x] - v[y, x + 1]) ** 2
            if y + 1 < H:
                w = 0.5 if x in (0, W - 1) else 1.0
                e += w * (v[y, x] - v[y + 1, x]) ** 2
    return e


def J_independent(P, b, u):
    m = triangles_touching(P.W, P.H) * P.h ** 2 / 6.0
    J = 0.0
    for i in range(P.N):
        mass_term = (m * u[i] ** 2).sum() / P.tau
        J += 0.5 * (mass_term + P.eps * edge_energy(u[i])) - (b[i] * u[i]).sum()
    return J


@pytest.mark.parametrize("W,H,N,pixel", [(2, 2, 2, True), (7, 5, 3, False), (12, 9, 4, True),
                                         (16, 16, 5, False), (5, 11, 8, True)])
def test_objective_matches_independent_quadratic(orc, W, H, N, pixel):
    h = 1.0 if pixel else 1.0 / (max(W, H) - 1)
    P = orc.Params(H=H, W=W, C=3, N=N, h=h, eps=2.0 * h, lam=50.0, tau=4.0 * h * h)
    rng = np.random.default_rng(W * 100 + H)
    for _ in range(3):
        u = rng.normal(0.3, 1.0, (N, H, W))
        b = rng.normal(0.0, 1.0, (N, H, W)) * h * h
        J = orc.objective(P, b, u)
        ref = J_independent(P, b, u)
        assert abs(J - ref) <= 1e-12 * max(1.0, abs(ref)), (J, ref)


def test_objective_separates_its_terms(orc):
    """Each of the three terms on its own: a constant field has no stiffness
    energy; b = 0 leaves the quadratic; u = 0 gives 0 whatever b."""
    W, H, N = 9, 6, 3
    P = orc.Params(H=H, W=W, C=3, N=N, h=0.5, eps=0.7, lam=1.0, tau=0.3)
    area = (W - 1) * (H - 1) * P.h ** 2
    u = np.full((N, H, W), 0.25)
    b = np.zeros_like(u)
    # (1/2) sum_i (0.25^2) * area / tau
    assert abs(orc.objective(P, b, u) - 0.5 * N * 0.0625 * area / P.tau) < 1e-13
    b = np.ones_like(u)
    ref = 0.5 * N * 0.0625 * area / P.tau - 0.25 * b.sum()
    assert abs(orc.objective(P, b, u) - ref) < 1e-12
    assert orc.objective(P, b, np.zeros_like(u)) == 0.0
