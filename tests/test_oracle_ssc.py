"""Pins for the oracle's subspace-correction iteration over all basis functions
(Section "Multigrid Solution", with the Gibbs correction of Section "Gibbs
Space Constraint Pseudocode").

  * each coarse basis function, as the oracle builds it by prolongation, is the
    P1 hat of its level's triangulation written out in closed form, and each
    level's functions sum to one at every finest node;
  * on the nodal functions the update is the projected block Gauss-Seidel
    update, so one iteration with one level is one lexicographic sweep (the
    corrections sum to zero, so they keep each node's sum: the start must lie
    on the simplices in FP64);
  * one update along a coarse function is the constrained minimiser of the step
    objective along that function, checked against scipy's SLSQP;
  * the update keeps u on the product of simplices, never raises the objective,
    and iterated to convergence it reaches the unique minimiser that the
    independent Gauss-Seidel / truncated multigrid path reaches.
"""
import numpy as np
import pytest
import scipy.optimize as so

from paper_0710_0736_amd import synth
from test_oracle_step import H_dense, J_of, params


def hat(W, H, s, X, Y, Wc, Hc):
    """P1 hat of coarse node (X, Y) on a lattice of spacing s whose cells are
    split along the (x,y)-(x+1,y+1) diagonal; finest nodes past the last coarse
    row or column take the value on it."""
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            dx = min(x / s, Wc - 1) - X
            dy = min(y / s, Hc - 1) - Y
            if dx * dy >= 0:
                v = 1 - max(abs(dx), abs(dy))
            else:
                v = 1 - abs(dx) - abs(dy)
            out[y, x] = max(v, 0.0)
    return out


def sides(W, H, L):
    out = [(W, H)]
    for _ in range(L - 1):
        W, H = (W + 1) // 2, (H + 1) // 2
        out.append((W, H))
    return out


@pytest.mark.parametrize("W,H,L", [(9, 9, 3), (12, 7, 3), (17, 10, 4)])
def test_basis_functions_are_coarse_hats(orc, W, H, L):
    P = params(orc, W, H, 3, pixel=True, levels=L)
    for l, (Wc, Hc) in enumerate(sides(W, H, L)):
        total = np.zeros((H, W))
        for q in range(Wc * Hc):
            eta = orc.basis(P, l, q)
            Y, X = divmod(q, Wc)
            np.testing.assert_allclose(eta, hat(W, H, 2 ** l, X, Y, Wc, Hc), atol=1e-15)
            assert eta[min(Y * 2 ** l, H - 1), min(X * 2 ** l, W - 1)] == 1.0
            total += eta
        np.testing.assert_allclose(total, 1.0, atol=1e-14)


def test_one_level_iteration_is_a_gauss_seidel_sweep(orc):
    W, H, N = 11, 8, 4
    P = params(orc, W, H, N, pixel=True, levels=1, max_cycles=1, tol=0.0)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=3)
    u0 = synth.random_simplex_field(N, H, W, seed=3).astype(np.float64)
    u0 /= u0.sum(0)  # on the simplices in FP64: the corrections keep each node's sum
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    u_gs, _ = orc.solve_qp(P, b, u0)
    P.ssc = True
    u_ssc, st = orc.solve_qp(P, b, u0)
    assert st["cycles"] == 1 and st["nonmonotone"] == 0
    np.testing.assert_allclose(u_ssc, u_gs, atol=1e-14)


def random_problem(orc, W, H, N, L, seed, sparse_u=True):
    P = params(orc, W, H, N, pixel=True, levels=L, lam=100.0)
    rng = np.random.default_rng(seed)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=seed)
    u = synth.random_simplex_field(N, H, W, seed=seed).astype(np.float64)
    u /= u.sum(0)
    if sparse_u:  # some components exactly zero, so bounds bind
        u = np.where(rng.random(u.shape) < 0.3, 0.0, u)
        u[0] += 1e-3
        u /= u.sum(0, keepdims=True)
    c, _ = orc.colour_means(P, img, u)
    b = orc.rhs(P, img, u, c)
    return P, u, b


@pytest.mark.parametrize("seed,l,q", [(0, 1, 4), (1, 1, 0), (2, 2, 4), (3, 1, 8), (4, 2, 0)])
def test_update_is_constrained_minimiser_along_basis_function(orc, seed, l, q):
    W, H, N = 9, 9, 3
    P, u, b = random_problem(orc, W, H, N, 3, seed)
    eta = orc.basis(P, l, q).ravel()
    Hm = H_dense(orc, P)
    uf = u.reshape(N, -1)
    bf = b.reshape(N, -1)

    def J(a):
        return J_of(Hm, bf, uf + np.outer(a, eta))

    sup = eta > 0
    cons = [{"type": "eq", "fun": lambda a: a.sum()}]
    for i in range(N):
        cons.append({"type": "ineq", "fun": lambda a, i=i: uf[i, sup] + a[i] * eta[sup]})
    ref = so.minimize(J, np.zeros(N), constraints=cons, method="SLSQP",
                      options={"ftol": 1e-15, "maxiter": 500})
    u_new, raised = orc.ssc_update(P, l, q, b, u)
    assert not raised
    # the update is u + alpha eta: recover alpha where eta = 1
    k = int(np.argmax(eta))
    alpha = u_new.reshape(N, -1)[:, k] - uf[:, k]
    np.testing.assert_allclose(u_new.reshape(N, -1), np.maximum(uf + np.outer(alpha, eta), 0.0), atol=1e-14)
    assert J(alpha) <= ref.fun + 1e-9 * abs(ref.fun)
    np.testing.assert_allclose(alpha, ref.x, atol=1e-6)


def test_updates_stay_feasible_and_monotone(orc):
    W, H, N, L = 13, 11, 4, 3
    P, u, b = random_problem(orc, W, H, N, L, 7)
    J0 = orc.objective(P, b, u)
    Wc = [s[0] * s[1] for s in sides(W, H, L)]
    for l in range(L - 1, -1, -1):
        for q in range(Wc[l]):
            u, raised = orc.ssc_update(P, l, q, b, u)
            assert not raised
            J1 = orc.objective(P, b, u)
            assert J1 <= J0 + 1e-12 * abs(J0)
            J0 = J1
            assert u.min() >= 0.0
            np.testing.assert_allclose(u.sum(0), 1.0, atol=1e-13)


@pytest.mark.parametrize("W,H,N,L,seed", [(24, 20, 3, 3, 0), (33, 33, 4, 0, 1)])
def test_iteration_reaches_the_unique_minimiser(orc, W, H, N, L, seed):
    P = params(orc, W, H, N, pixel=True, levels=L, lam=100.0, tol=1e-12)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=seed)
    u0 = synth.random_simplex_field(N, H, W, seed=seed).astype(np.float64)
    u0 /= u0.sum(0)
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    u_mg, st_mg = orc.solve_qp(P, b, u0)
    P.ssc = True
    u_ssc, st = orc.solve_qp(P, b, u0)
    assert st["converged"] and st_mg["converged"]
    assert st["nonmonotone"] == 0
    # both within tol / (1 - q) of the minimiser; q <= 0.98 in pixel units
    np.testing.assert_allclose(u_ssc, u_mg, atol=1e-10)
    # active components exist, so the bounds of the coarse updates were exercised
    assert (u_ssc == 0).mean() > 0.05
