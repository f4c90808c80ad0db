"""Pins of the data pre-pass oracle (no GPU).

* refinement: the rule of Section "Data Projection" checked node by node (every
  node a refinement creates equals one of its lattice neighbours; old nodes
  keep their values; no new values appear), lattice sizes and their nesting
  into the multigrid hierarchy, and sampling as its left inverse;
* colour space: invariants of CIE L*a*b* (white -> L* = 100, a* = b* = 0;
  black -> 0; every grey -> a* = b* = 0; L* increasing along the greys),
  continuity of both piecewise definitions at their knots, and the published
  L*a*b* of the sRGB primaries.
"""
import numpy as np
import pytest

from oracle import data as od

NEIGHBOURS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


@pytest.mark.parametrize("W,H,P", [(2, 2, 1), (5, 3, 2), (7, 9, 3)])
def test_refine_once_follows_the_injection_rule(W, H, P):
    rng = np.random.default_rng(W * H)
    a = rng.integers(0, 1000, size=(P, H, W)).astype(np.float64)  # distinct-ish values
    f = od.refine_once(a)
    assert f.shape == (P, 2 * H - 1, 2 * W - 1)
    assert np.array_equal(f[:, ::2, ::2], a)
    for c in range(P):
        for Y in range(2 * H - 1):
            for X in range(2 * W - 1):
                if X % 2 == 0 and Y % 2 == 0:
                    continue
                # a created node carries the value of one of its lattice neighbours
                vals = [f[c, Y + dy, X + dx] for dy, dx in NEIGHBOURS
                        if 0 <= Y + dy < 2 * H - 1 and 0 <= X + dx < 2 * W - 1]
                assert f[c, Y, X] in vals, (c, X, Y)
    assert set(np.unique(f)) <= set(np.unique(a))


@pytest.mark.parametrize("W,H,r", [(2, 2, 0), (3, 2, 1), (6, 5, 3), (17, 9, 2)])
def test_refine_sizes_nesting_and_sampling(W, H, r):
    rng = np.random.default_rng(r)
    a = rng.random((2, H, W))
    f = od.refine(a, r)
    Wf, Hf = (W - 1) * 2 ** r + 1, (H - 1) * 2 ** r + 1
    assert f.shape == (2, Hf, Wf)
    # the multigrid coarsening ceil(side / 2) of the refined lattice reaches the pixel lattice
    w, h = Wf, Hf
    for _ in range(r):
        w, h = (w + 1) // 2, (h + 1) // 2
    assert (w, h) == (W, H)
    assert np.array_equal(od.sample(f, r), a)
    # piecewise constant: node (X, Y) holds pixel (X >> r, Y >> r)
    Y, X = np.mgrid[0:Hf, 0:Wf]
    assert np.array_equal(f, a[:, Y >> r, X >> r])


def test_lab_white_black_and_greys():
    g = np.linspace(0.0, 1.0, 101)
    rgb = np.stack([g, g, g])
    lab = od.srgb_to_lab(rgb) * 100.0
    assert abs(lab[0, -1] - 100.0) < 1e-9 and np.abs(lab[1:, -1]).max() < 1e-9
    assert np.abs(lab[:, 0]).max() < 1e-9
    assert np.abs(lab[1:]).max() < 1e-9
    assert np.all(np.diff(lab[0]) > 0)
    ab = od.srgb_to_lab(rgb, ab_only=True)
    assert ab.shape == (2, 101) and np.array_equal(ab, lab[1:] / 100.0)


def test_lab_piecewise_definitions_are_continuous_at_their_knots():
    k = 0.04045  # the sRGB transfer curve's knot
    assert abs(k / 12.92 - ((k + 0.055) / 1.055) ** 2.4) < 1e-7
    lo, hi = od.srgb_to_linear([k, k + 1e-9])
    assert abs(hi - lo) < 1e-8
    d = 6.0 / 29.0  # the CIE companding knot: value and slope match
    t = d ** 3
    assert abs(od.cie_f(t) - od.cie_f(t * (1 + 1e-9))) < 1e-8
    slope_lin = 1.0 / (3 * d * d)
    slope_cbrt = (1.0 / 3.0) * t ** (-2.0 / 3.0)
    assert abs(slope_lin - slope_cbrt) < 1e-9


def test_lab_of_the_srgb_primaries():
    # L*a*b* (D65) of pure sRGB red, green and blue as tabulated in the
    # colour-science literature; the 4-digit matrix keeps them within 0.05
    ref = {(1, 0, 0): (53.24, 80.09, 67.20), (0, 1, 0): (87.73, -86.18, 83.18),
           (0, 0, 1): (32.30, 79.19, -107.86)}
    for rgb, want in ref.items():
        got = od.srgb_to_lab(np.array(rgb, dtype=np.float64).reshape(3, 1))[:, 0] * 100.0
        assert np.abs(got - np.array(want)).max() < 0.05, (rgb, got)
    # middle grey: the transfer curve maps 0.5 to 0.2140 (linear light)
    assert abs(od.srgb_to_linear(0.5) - 0.2140) < 1e-4


def test_mass_matrix_and_mass_average():
    W, H, h = 7, 5, 0.4
    M = od.mass_matrix(W, H, h).toarray()
    assert np.allclose(M, M.T)
    assert np.linalg.eigvalsh(M).min() > 0
    # row sums: the lumped mass h^2 w of the node classes (interior 1, edge 1/2,
    # corners (0,0)/(W-1,H-1) 1/3, the other two 1/6); total = domain area
    m = M.sum(axis=1).reshape(H, W) / h ** 2
    assert np.allclose(m[1:-1, 1:-1], 1.0) and np.allclose(m[0, 1:-1], 0.5) and np.allclose(m[1:-1, 0], 0.5)
    assert np.isclose(m[0, 0], 1 / 3) and np.isclose(m[-1, -1], 1 / 3)
    assert np.isclose(m[0, -1], 1 / 6) and np.isclose(m[-1, 0], 1 / 6)
    assert np.isclose(M.sum(), ((W - 1) * h) * ((H - 1) * h))
    # constants are kept everywhere, linear functions at every interior node
    # (the six triangles around it are symmetric about it)
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.stack([np.full((H, W), 0.3), 0.2 * X - 0.1 * Y + 0.05])
    av = od.mass_average(img, h)
    assert np.allclose(av[0], 0.3)
    assert np.allclose(av[1][1:-1, 1:-1], img[1][1:-1, 1:-1])
    assert not np.allclose(av[1], img[1])  # the boundary sees a one-sided average


def test_consistent_mass_fitting_is_the_lumped_solver_on_the_mass_average():
    """Consistent-mass fitting (gradient lambda M F_i, means u_i.M I / u_i.M 1) gives
    the same step as the lumped oracle on I~ = M I / m: the right-hand sides differ
    by a term common to all phases at each node, and the means agree."""
    import oracle as orc
    from paper_0710_0736_amd import synth
    W, H, N, C, h = 9, 7, 3, 2, 0.3
    P = orc.Params(H=H, W=W, C=C, N=N, h=h, eps=2 * h, lam=20.0, tau=(2 * h) ** 2, levels=1, tol=1e-12)
    rng = np.random.default_rng(5)
    img = rng.random((C, H, W))
    un = synth.random_simplex_field(N, H, W, seed=6).astype(np.float64)
    M = od.mass_matrix(W, H, h)
    m = np.asarray(M.sum(axis=1)).ravel()
    # consistent-mass means and right-hand side, from their definitions
    MI = np.stack([M @ img[k].ravel() for k in range(C)])
    c_cons = np.array([[un[i].ravel() @ MI[k] / (un[i].ravel() @ m) for k in range(C)] for i in range(N)])
    a = 1.0 / P.tau + 2.0 / P.eps
    b_cons = np.empty((N, H, W))
    for i in range(N):
        F = sum((img[k] - c_cons[i, k]) ** 2 for k in range(C)).ravel()
        b_cons[i] = (m * a * un[i].ravel() - P.lam * (M @ F)).reshape(H, W)
    # the lumped oracle on the mass average
    Ia = od.mass_average(img, h)
    c_red, _ = orc.colour_means(P, Ia, un)
    assert np.abs(c_red - c_cons).max() < 1e-12
    b_red = orc.rhs(P, Ia, un, c_red)
    d = b_cons - b_red
    assert np.abs(d - d[0:1]).max() < 1e-10 * np.abs(b_cons).max()
    u_cons, s1 = orc.solve_qp(P, b_cons, un)
    u_red, s2 = orc.solve_qp(P, b_red, un)
    assert s1["converged"] and s2["converged"]
    assert np.abs(u_cons - u_red).max() < 1e-9


def test_simplex_average_invariants_and_relation_to_the_mass_matrix():
    """Projection by simplex: constants and (at interior nodes) linear functions
    are kept, and per triangle (I_p + I_a + I_b) / 9 = (4/3) (2 I_p + I_a + I_b) / 12
    - I_p / 9, so the by-simplex value is (4/3) (M I) / m - I / 3 with M the
    consistent mass matrix assembled independently."""
    W, H, h = 8, 6, 0.7
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.stack([np.full((H, W), -0.4), 0.3 * X + 0.2 * Y - 1.0])
    sa = od.simplex_average(img, h)
    assert np.allclose(sa[0], -0.4)
    assert np.allclose(sa[1][1:-1, 1:-1], img[1][1:-1, 1:-1])
    rng = np.random.default_rng(11)
    img = rng.random((3, H, W))
    sa = od.simplex_average(img, h)
    ca = od.mass_average(img, h)
    np.testing.assert_allclose(sa, 4.0 / 3.0 * ca - img / 3.0, atol=1e-14)


def test_simplex_projection_fitting_is_the_lumped_solver_on_the_simplex_average():
    """Fitting with the image replaced by its element values I_t (projection by
    simplex): the fidelity gradient sum_t (I_t - c_i)^2 |t| / 3 at each node and
    the means int u_i I / int u_i, built element by element, give the same step
    as the lumped oracle on the simplex average (the right-hand sides differ by a
    term common to all phases at each node)."""
    import oracle as orc
    from paper_0710_0736_amd import synth
    W, H, N, C, h = 8, 7, 3, 2, 0.3
    P = orc.Params(H=H, W=W, C=C, N=N, h=h, eps=2 * h, lam=20.0, tau=(2 * h) ** 2, levels=1, tol=1e-12)
    rng = np.random.default_rng(7)
    img = rng.random((C, H, W))
    un = synth.random_simplex_field(N, H, W, seed=8).astype(np.float64)
    area = h * h / 2.0
    tris = []
    for cy in range(H - 1):
        for cx in range(W - 1):
            tris.append(((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)))
            tris.append(((cx, cy), (cx, cy + 1), (cx + 1, cy + 1)))
    It = np.array([[sum(img[k, y, x] for x, y in t) / 3.0 for k in range(C)] for t in tris])
    m = np.zeros((H, W))
    for t in tris:
        for x, y in t:
            m[y, x] += area / 3.0
    # means: int u_i I = sum_t I_t int_t u_i, int_t u_i = |t| (u_a + u_b + u_c) / 3
    c_el = np.zeros((N, C))
    for i in range(N):
        mass = (m * un[i]).sum()
        for ti, t in enumerate(tris):
            ut = sum(un[i, y, x] for x, y in t) / 3.0
            c_el[i] += It[ti] * area * ut
        c_el[i] /= mass
    a = 1.0 / P.tau + 2.0 / P.eps
    b_el = np.empty((N, H, W))
    for i in range(N):
        g = np.zeros((H, W))
        for ti, t in enumerate(tris):
            f = ((It[ti] - c_el[i]) ** 2).sum()
            for x, y in t:
                g[y, x] += area / 3.0 * f
        b_el[i] = m * a * un[i] - P.lam * g
    Is = od.simplex_average(img, h)
    c_red, _ = orc.colour_means(P, Is, un)
    assert np.abs(c_red - c_el).max() < 1e-12
    b_red = orc.rhs(P, Is, un, c_red)
    d = b_el - b_red
    assert np.abs(d - d[0:1]).max() < 1e-10 * np.abs(b_el).max()
    u_el, s1 = orc.solve_qp(P, b_el, un)
    u_red, s2 = orc.solve_qp(P, b_red, un)
    assert s1["converged"] and s2["converged"]
    assert np.abs(u_el - u_red).max() < 1e-9
