"""Pins for the oracle's colour means, right-hand side and per-step solve.

Every step solves a strictly convex quadratic program over a product of
simplices, so its answer is unique and can be reached by any convergent
method.  The oracle's Gauss-Seidel / multigrid answer is checked against:
  * accelerated projected gradient (FISTA) with the sort-based projection;
  * scipy's SLSQP on the same objective (library QP);
  * the N = 2 reduction to a box-constrained QP (L-BFGS-B);
  * the closed-form linear solve when no constraint is active (spsolve);
  * the KKT conditions of the simplex-constrained QP;
and the right-hand side is checked against finite-difference gradients of the
independently pinned discrete energy.  Colour means are checked on exact
piecewise-constant data and the empty-phase rule.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_0710_0736_amd import synth
from test_oracle_assembly import dense_A, triangles_per_node
from test_oracle_projection import proj_sort


def params(orc, W, H, N, C=3, pixel=False, lam=50.0, **kw):
    h = 1.0 if pixel else 1.0 / (max(W, H) - 1)
    return orc.Params(H=H, W=W, C=C, N=N, h=h, eps=2 * h, lam=lam, tau=4 * h * h, **kw)


def H_dense(orc, P):
    m, s = orc.assemble(P.W, P.H, P.h)
    return np.diag(m.ravel()) / P.tau + P.eps * dense_A(s)


def small_problem(orc, W, H, N, pixel, seed, lam=50.0):
    P = params(orc, W, H, N, pixel=pixel, lam=lam, tol=1e-13)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=seed)
    u0 = synth.random_simplex_field(N, H, W, seed=seed)
    c, _ = orc.colour_means(P, img, u0)
    b = orc.rhs(P, img, u0, c)
    return P, img, u0, b


def J_of(Hm, b, u):
    return sum(0.5 * u[i] @ Hm @ u[i] - b[i] @ u[i] for i in range(len(u)))


def fista(Hm, b, N, n, iters=20000):
    """Accelerated projected gradient on the product of simplices."""
    L = np.linalg.eigvalsh(Hm).max()
    x = np.full((N, n), 1.0 / N)
    yk, t = x.copy(), 1.0
    for _ in range(iters):
        g = np.stack([Hm @ yk[i] - b[i] for i in range(N)])
        z = yk - g / L
        xn = np.stack([proj_sort(z[:, p]) for p in range(n)], 1)
        tn = 0.5 * (1 + np.sqrt(1 + 4 * t * t))
        yk = xn + (t - 1) / tn * (xn - x)
        if np.abs(xn - x).max() < 1e-15:
            x = xn
            break
        x, t = xn, tn
    return x


@pytest.mark.parametrize("N,pixel", [(2, False), (3, True), (4, True), (2, True)])
def test_bruteforce_4x4(orc, N, pixel):
    W = H = 4
    P, img, u0, b = small_problem(orc, W, H, N, pixel, seed=N, lam=5.0)
    Hm = H_dense(orc, P)
    n = W * H
    bf = b.reshape(N, n)
    u, st = orc.solve_qp(P, b, u0)
    assert st["converged"] and st["nonmonotone"] == 0
    uf = fista(Hm, bf, N, n)
    assert np.abs(u.reshape(N, n) - uf).max() < 1e-9
    # SLSQP (library QP) agrees in objective and solution
    cons = [{"type": "eq", "fun": lambda z, p=p: z.reshape(N, n)[:, p].sum() - 1.0} for p in range(n)]
    res = so.minimize(lambda z: J_of(Hm, bf, z.reshape(N, n)), np.full(N * n, 1.0 / N),
                      jac=lambda z: np.concatenate([Hm @ z.reshape(N, n)[i] - bf[i] for i in range(N)]),
                      bounds=[(0, None)] * (N * n), constraints=cons, method="SLSQP",
                      options={"ftol": 1e-15, "maxiter": 2000})
    assert J_of(Hm, bf, u.reshape(N, n)) <= res.fun + 1e-9 * abs(res.fun)
    assert np.abs(u.reshape(N, n) - res.x.reshape(N, n)).max() < 1e-5


def test_two_phase_box_qp(orc):
    # with N = 2, u2 = 1 - u1 and the step is a box QP in u1 with Hessian 2H
    W, H = 9, 7
    P, img, u0, b = small_problem(orc, W, H, 2, True, seed=7, lam=20.0)
    Hm = H_dense(orc, P)
    n = W * H
    bf = b.reshape(2, n)
    q = bf[0] - bf[1] + Hm @ np.ones(n)
    res = so.minimize(lambda z: z @ Hm @ z - q @ z, np.full(n, 0.5), jac=lambda z: 2 * Hm @ z - q,
                      bounds=[(0, 1)] * n, method="L-BFGS-B",
                      options={"ftol": 1e-16, "gtol": 1e-13, "maxiter": 20000})
    u, st = orc.solve_qp(P, b, u0)
    assert 0 < (u[0] == 0).mean() + (u[0] == 1).mean() < 1  # some bounds active, some not
    assert np.abs(u[0].ravel() - res.x).max() < 1e-6


def test_interior_step_is_linear_solve(orc):
    # unit-square scale: nothing becomes active, so u_i = H^-1 (b_i - mean_j b_j) + 1/N
    W, H, N = 24, 20, 3
    P, img, u0, b = small_problem(orc, W, H, N, False, seed=3, lam=100.0)
    u, st = orc.solve_qp(P, b, u0)
    assert (u > 1e-3).all()
    Hs = sp.csc_matrix(H_dense(orc, P))
    bf = b.reshape(N, -1)
    bbar = bf.mean(0)
    for i in range(N):
        ui = spla.spsolve(Hs, bf[i] - bbar) + 1.0 / N
        assert np.abs(ui - u[i].ravel()).max() < 1e-9


@pytest.mark.parametrize("levels", [1, 0])
def test_kkt_of_step(orc, levels):
    W, H, N = 20, 16, 4
    P, img, u0, b = small_problem(orc, W, H, N, True, seed=11, lam=30.0)
    P.levels = levels
    u, st = orc.solve_qp(P, b, u0)
    G = (orc.apply_H(P, u) - b).reshape(N, -1)  # gradient of J
    uf = u.reshape(N, -1)
    scale = np.abs(G).max()
    active_any = False
    for p in range(W * H):
        free = uf[:, p] > 0
        mu = G[free, p].mean()
        assert np.abs(G[free, p] - mu).max() < 1e-7 * scale
        assert (G[~free, p] >= mu - 1e-7 * scale).all()
        active_any |= (~free).any()
    assert active_any


def test_multigrid_and_gauss_seidel_agree(orc):
    w = synth.pixel_twin(synth.VORONOI1024, 48)
    img, u0, _ = w.make(2)
    P0 = orc.Params.from_workload(w, levels=0, tol=1e-11)
    P1 = orc.Params.from_workload(w, levels=1, tol=1e-11)
    u0n, c0, s0 = orc.step(P0, img, u0)
    u1n, c1, s1 = orc.step(P1, img, u0)
    assert s0["converged"] and s1["converged"] and s0["nonmonotone"] == 0
    assert s0["cycles"] < s1["cycles"]
    assert np.abs(u0n - u1n).max() < 1e-9


def test_colour_means_exact_on_piecewise_constant(orc):
    W, H, N = 17, 13, 4
    rng = np.random.default_rng(0)
    lab = rng.integers(0, N, (H, W))
    lab[0, 0] = 0
    col = rng.uniform(0, 1, (N, 3))
    img = col[lab].transpose(2, 0, 1)
    P = params(orc, W, H, N)
    c, empty = orc.colour_means(P, img, synth.one_hot(lab, N))
    assert not empty
    assert np.allclose(c, col, atol=1e-14)
    # I + t shifts every mean by t; a channel permutation permutes the means
    u = synth.random_simplex_field(N, H, W, seed=1)
    c1, _ = orc.colour_means(P, img, u)
    c2, _ = orc.colour_means(P, img + 0.25, u)
    assert np.allclose(c2, c1 + 0.25, atol=1e-14)
    c3, _ = orc.colour_means(P, img[[2, 0, 1]], u)
    assert np.allclose(c3, c1[:, [2, 0, 1]], atol=1e-15)
    # mass-weighted mean with the triangle-count weights
    m = triangles_per_node(W, H).ravel()
    uf, If = u.reshape(N, -1), img.reshape(3, -1)
    assert np.allclose(c1, (uf * m) @ If.T / (uf * m).sum(1)[:, None], atol=1e-13)


def test_empty_phase_rule(orc):
    W, H, N = 8, 8, 3
    img, _ = synth.voronoi_image(W, H, 2, 0.05, seed=0)
    u = synth.one_hot(np.zeros((H, W), np.int64), N)
    P = params(orc, W, H, N)
    c, empty = orc.colour_means(P, img, u)
    assert empty
    m = triangles_per_node(W, H).ravel()
    mean_col = (img.reshape(3, -1) * m).sum(1) / m.sum()
    assert np.allclose(c[1], mean_col) and np.allclose(c[2], mean_col)
    cp = np.arange(9.0).reshape(3, 3)
    c, empty = orc.colour_means(P, img, u, cp)
    assert np.allclose(c[1:], cp[1:]) and np.allclose(c[0], mean_col)


def test_rhs_is_energy_linearisation(orc):
    """b = M un / tau - grad(concave + fitting energy)(un) up to a per-node constant.

    The fitting part uses c(u) inside the energy; its gradient at fixed c equals
    the full gradient because c(u) minimises the fitting term over c.
    """
    W, H, N = 7, 6, 3
    P = params(orc, W, H, N, pixel=True, lam=3.0)
    img, _ = synth.voronoi_image(W, H, N, 0.1, seed=4)
    un = synth.random_simplex_field(N, H, W, seed=4).astype(np.float64)
    c, _ = orc.colour_means(P, img, un)
    b = orc.rhs(P, img, un, c)
    m, _ = orc.assemble(W, H, P.h)

    def E12(u):
        _, parts = orc.energy(P, img, u)
        return parts[1] + parts[2]

    g = np.zeros_like(un)
    d = 1e-6
    for k in range(un.size):
        e = np.zeros(un.size)
        e[k] = d
        e = e.reshape(un.shape)
        g.flat[k] = (E12(un + e) - E12(un - e)) / (2 * d)
    expect = m[None] * un / P.tau - g
    diff = (b - expect).reshape(N, -1)
    assert np.abs(diff - diff.mean(0)).max() < 1e-6


def test_natural_residual_sees_a_single_node_perturbation(orc):
    """rho(u) = max |Pi(y_p(u)) - u_p|: y_p does not involve u_p, so moving a
    converged solution by delta at one node (feasibly, between two free
    components) gives rho = delta there, while the neighbours only see
    kappa * delta < delta."""
    W, H, N = 12, 10, 3
    P, img, u0, b = small_problem(orc, W, H, N, False, seed=21, lam=10.0)
    u, st = orc.solve_qp(P, b, u0)
    assert orc.residual(P, b, u) < 1e-12
    y, x = 4, 6
    i, j = np.argsort(u[:, y, x])[-2:]
    d = 0.25 * min(u[i, y, x], u[j, y, x])
    up = u.copy()
    up[i, y, x] += d
    up[j, y, x] -= d
    assert orc.residual(P, b, up) == pytest.approx(d, rel=1e-9)
