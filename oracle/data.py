"""FP64 CPU oracle for the data pre-passes: refined lattices and colour spaces.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's checks,
never by the product path.  Plain numpy, no code shared with the HIP kernels.

Parity status: pinned by ``tests/test_oracle_data.py`` (the paper's injection
rule checked node by node, invariants of the colour transform, continuity at
its knots, published values of the sRGB primaries, the consistent and
by-simplex projections against each other and against steps assembled from
their definitions); none is "parity unpinned".
"""
from __future__ import annotations

import numpy as np


def refine_once(a: np.ndarray) -> np.ndarray:
    """One uniform refinement of the data on a lattice (Section "Data Projection").

    ``a`` is [planes][H][W]; the refined lattice has (2H - 1) x (2W - 1) nodes,
    old node (x, y) on new node (2x, 2y).  Every new node (an edge midpoint
    along x or y, or the midpoint of the cell diagonal) is given the value of
    one of its neighbours, never an interpolated value: here the old node at
    its lower-left, so no new values (and no new gradients) appear.
    """
    a = np.asarray(a, dtype=np.float64)
    P, H, W = a.shape
    f = np.empty((P, 2 * H - 1, 2 * W - 1))
    f[:, 0::2, 0::2] = a                       # old nodes keep their values
    f[:, 0::2, 1::2] = a[:, :, :-1]            # midpoints along x: left neighbour
    f[:, 1::2, 0::2] = a[:, :-1, :]            # midpoints along y: lower neighbour
    f[:, 1::2, 1::2] = a[:, :-1, :-1]          # cell-diagonal midpoints: lower-left corner
    return f


def refine(a: np.ndarray, r: int) -> np.ndarray:
    """r successive refinements (Section "Determination of Natural Scales")."""
    out = np.asarray(a, dtype=np.float64)
    for _ in range(r):
        out = refine_once(out)
    return out


def sample(f: np.ndarray, r: int) -> np.ndarray:
    """The values of a refined field at the original lattice's nodes."""
    s = 1 << r
    return np.asarray(f, dtype=np.float64)[:, ::s, ::s]


# sRGB (IEC 61966-2-1): transfer curve and the matrix from linear RGB to CIE XYZ
# of the sRGB primaries with the D65 white.
SRGB_TO_XYZ = np.array([[0.4124, 0.3576, 0.1805],
                        [0.2126, 0.7152, 0.0722],
                        [0.0193, 0.1192, 0.9505]])


def srgb_to_linear(v):
    v = np.asarray(v, dtype=np.float64)
    return np.where(v <= 0.04045, v / 12.92, ((v + 0.055) / 1.055) ** 2.4)


def cie_f(t):
    """The CIE 1976 companding function: cube root above (6/29)^3, linear below."""
    t = np.asarray(t, dtype=np.float64)
    d = 6.0 / 29.0
    return np.where(t > d ** 3, np.cbrt(t), t / (3 * d * d) + 4.0 / 29.0)


def srgb_to_lab(rgb, ab_only: bool = False) -> np.ndarray:
    """sRGB [3][...] in [0, 1] -> CIE L*a*b* / 100 (or a*b* / 100).

    The white point is the XYZ of RGB (1, 1, 1) (the matrix's row sums), the
    choice under which white and the greys have a* = b* = 0.
    """
    rgb = np.asarray(rgb, dtype=np.float64)
    lin = srgb_to_linear(rgb)
    xyz = np.tensordot(SRGB_TO_XYZ, lin, axes=1)
    white = SRGB_TO_XYZ.sum(axis=1)
    fx, fy, fz = (cie_f(xyz[k] / white[k]) for k in range(3))
    L = 116.0 * fy - 16.0
    a = 500.0 * (fx - fy)
    b = 200.0 * (fy - fz)
    out = np.stack([a, b]) if ab_only else np.stack([L, a, b])
    return out / 100.0


def mass_matrix(W: int, H: int, h: float = 1.0):
    """Consistent P1 mass matrix M_pq = (eta_p, eta_q) of the W x H lattice, every
    cell split along its (x, y)-(x+1, y+1) diagonal (Section "Data Projection",
    the standard mass matrix).  Assembled element by element: a triangle of
    area |T| adds |T|/6 to each diagonal entry of its vertices and |T|/12 to
    each pair.  Returns a scipy CSR matrix over nodes p = y W + x."""
    import scipy.sparse as sp
    rows, cols, vals = [], [], []
    area = h * h / 2.0
    for cy in range(H - 1):
        for cx in range(W - 1):
            for tri in (((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)),
                        ((cx, cy), (cx, cy + 1), (cx + 1, cy + 1))):
                for a in tri:
                    for b in tri:
                        rows.append(a[1] * W + a[0])
                        cols.append(b[1] * W + b[0])
                        vals.append(area / 6.0 if a == b else area / 12.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(W * H, W * H))


def mass_average(img: np.ndarray, h: float = 1.0) -> np.ndarray:
    """The image as the consistent mass matrix sees it: (M I)_p / m_p per channel,
    with m_p = sum_q M_pq the lumped mass."""
    img = np.asarray(img, dtype=np.float64)
    C, H, W = img.shape
    M = mass_matrix(W, H, h)
    m = np.asarray(M.sum(axis=1)).ravel()
    return np.stack([(M @ img[k].ravel()) / m for k in range(C)]).reshape(C, H, W)


def simplex_average(img: np.ndarray, h: float = 1.0) -> np.ndarray:
    """The image as "projection by simplex" sees it (Section "Data Projection").

    The image enters only through its integral over each element, so it is
    replaced by one value per triangle, I_t = its integral over t divided by |t|:
    for the P1 interpolant of the nodal data, the mean of the three vertex
    values.  The load vector is (M I)_p = sum_{t at p} I_t <eta_p, 1>_t =
    sum_t I_t |t| / 3 (the basis functions sum to one on t), and the nodal value
    is (M I)_p / m_p with m_p = sum_t |t| / 3 the lumped mass.  Assembled
    element by element over the lattice cells, each split along its
    (x, y)-(x+1, y+1) diagonal.
    """
    img = np.asarray(img, dtype=np.float64)
    C, H, W = img.shape
    load = np.zeros((C, H, W))
    m = np.zeros((H, W))
    area = h * h / 2.0
    for cy in range(H - 1):
        for cx in range(W - 1):
            for tri in (((cx, cy), (cx + 1, cy), (cx + 1, cy + 1)),
                        ((cx, cy), (cx, cy + 1), (cx + 1, cy + 1))):
                It = sum(img[:, y, x] for x, y in tri) / 3.0
                for x, y in tri:
                    load[:, y, x] += area / 3.0 * It
                    m[y, x] += area / 3.0
    return load / m
