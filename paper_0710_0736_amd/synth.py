"""Seeded synthetic workloads for the vector-valued Allen-Cahn segmentation solver.

This module only draws random numbers and paints pictures: it holds none of the
method's arithmetic (no mass matrix, no colour means, no projection, no solver).
Both the HIP path's callers (benchmark, tests) and the FP64 oracle's tests take
their inputs from here, so both sides always see bit-identical arrays.

Conventions
-----------
* Arrays are structure-of-arrays: an image is ``[C][H][W]``, a phase field is
  ``[N][H][W]``, node ``(x, y)`` at flat index ``y * W + x``.
* Node ``(x, y)`` sits at the physical point ``(x*h, y*h)``.  The unit-square
  scale uses ``h = 1/(max(W, H) - 1)``; the "pixel-unit" twins use ``h = 1``.
* Every draw comes from its own PCG64 stream keyed by ``(seed, purpose)`` so
  that changing one ingredient never shifts another.  Everything is drawn in
  float64 and rounded to float32 exactly once.
* The paper's own images are not available; these stand in for them
  (piecewise-constant and piecewise-linear colour regions with Gaussian noise).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

# purpose keys of the independent random streams
_S_SITES, _S_COLOURS, _S_NOISE, _S_U0, _S_RAMP, _S_BATCH, _S_DIR = range(1, 8)


def _rng(seed: int, purpose: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(purpose), int(extra)]))


def unit_spacing(W: int, H: int) -> float:
    """Lattice spacing that maps the longer image side onto [0, 1]."""
    return 1.0 / (max(W, H) - 1)


def _coords(W: int, H: int, h: float):
    x = np.arange(W, dtype=np.float64) * h
    y = np.arange(H, dtype=np.float64) * h
    return np.meshgrid(x, y)  # each [H][W]


def _noisy(clean: np.ndarray, sigma: float, seed: int, clip: bool) -> np.ndarray:
    noise = _rng(seed, _S_NOISE).standard_normal(clean.shape)
    img = clean + sigma * noise
    if clip:
        img = np.clip(img, 0.0, 1.0)
    return img.astype(np.float32)


def disk_image(W: int = 64, H: int = 64, radius: float = 0.3,
               centre: Tuple[float, float] = (0.5, 0.5),
               fg: Tuple[float, ...] = (0.8, 0.2, 0.2), bg: Tuple[float, ...] = (0.1, 0.1, 0.7),
               sigma: float = 0.05, clip: bool = True, seed: int = 0):
    """A disk of colour ``fg`` on a ``bg`` background plus i.i.d. Gaussian noise.

    Returns ``(image [C][H][W] float32, labels [H][W] uint8)`` with label 1 inside.
    The disk geometry is fixed in physical units (unit-square scale by default).
    """
    X, Y = _coords(W, H, unit_spacing(W, H))  # geometry on the unit square
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 <= radius ** 2
    fg = np.asarray(fg, np.float64)
    bg = np.asarray(bg, np.float64)
    clean = np.where(inside[None], fg[:, None, None], bg[:, None, None])
    return _noisy(clean, sigma, seed, clip), inside.astype(np.uint8)


def voronoi_image(W: int, H: int, n_regions: int, sigma: float, seed: int = 0,
                  ramp: float = 0.0, clip: bool = False, channels: int = 3):
    """Voronoi partition from ``n_regions`` seeded sites with random colours.

    Sites are uniform on the image rectangle, region = nearest site (ties to the
    lowest index), colours uniform in [0, 1]^C.  With ``ramp > 0`` every region
    and channel gets an additional linear ramp centred at its site, with a
    uniformly random direction and a magnitude uniform in [0, ramp] per unit
    length of the unit-square scale.  Returns ``(image, labels)``.
    """
    hu = unit_spacing(W, H)
    X, Y = _coords(W, H, hu)
    r = _rng(seed, _S_SITES)
    sites = np.stack([r.uniform(0.0, (W - 1) * hu, n_regions),
                      r.uniform(0.0, (H - 1) * hu, n_regions)], axis=1)
    colours = _rng(seed, _S_COLOURS).uniform(0.0, 1.0, (n_regions, channels))
    best = np.full((H, W), np.inf)
    labels = np.zeros((H, W), np.int64)
    for k in range(n_regions):  # strict '<' keeps the lowest index on ties
        d = (X - sites[k, 0]) ** 2 + (Y - sites[k, 1]) ** 2
        closer = d < best
        labels[closer] = k
        best[closer] = d[closer]
    clean = colours[labels].transpose(2, 0, 1).copy()  # [C][H][W]
    if ramp > 0.0:
        rr = _rng(seed, _S_RAMP)
        ang = rr.uniform(0.0, 2 * np.pi, (n_regions, channels))
        mag = rr.uniform(0.0, ramp, (n_regions, channels))
        gx, gy = mag * np.cos(ang), mag * np.sin(ang)
        for c in range(channels):
            clean[c] += (gx[labels, c] * (X - sites[labels, 0])
                         + gy[labels, c] * (Y - sites[labels, 1]))
    return _noisy(clean, sigma, seed, clip), labels.astype(np.uint8)


def concentric_circles(W: int = 128, H: int = 128, levels=(0.25, 0.95, 0.55, 0.75),
                       background: float = 0.1, amplitude: float = 0.05, seed: int = 0):
    """Grayscale (C = 1) concentric rings at the given grey levels on a background.

    Grey levels, background and noise amplitude are the ones the paper quotes
    for its concentric-circle example; the radii are not given there and are
    chosen here as equal steps out to 0.4 of the unit square.  Noise is uniform
    in [-amplitude, amplitude].  Returns ``(image [1][H][W], labels)`` where
    label 0 is the background and label k the k-th ring from the outside.
    """
    X, Y = _coords(W, H, unit_spacing(W, H))
    rho = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    n = len(levels)
    radii = 0.4 * (1.0 - np.arange(n) / n)  # outer radius of each ring
    labels = np.zeros((H, W), np.int64)
    for k in range(n):
        labels[rho <= radii[k]] = k + 1
    grey = np.concatenate([[background], np.asarray(levels, np.float64)])
    clean = grey[labels][None]
    noise = _rng(seed, _S_NOISE).uniform(-amplitude, amplitude, clean.shape)
    return (clean + noise).astype(np.float32), labels.astype(np.uint8)


def random_simplex_field(N: int, H: int, W: int, seed: int = 0) -> np.ndarray:
    """Initial phase field: an independent Dirichlet(1, ..., 1) sample per node.

    ``e = -log(U)`` with ``U`` uniform on (0, 1] from PCG64, normalised per node
    in float64, rounded to float32 and normalised once more.
    """
    r = _rng(seed, _S_U0)
    e = -np.log1p(-r.random((N, H, W)))  # U in [0,1) -> 1-U in (0,1]
    u = e / e.sum(axis=0, keepdims=True)
    u32 = u.astype(np.float32)
    return (u32 / u32.sum(axis=0, keepdims=True, dtype=np.float64)).astype(np.float32)


def one_hot(labels: np.ndarray, N: int) -> np.ndarray:
    """``[N][H][W]`` float32 indicator of ``labels`` (values in 0..N-1)."""
    return (labels[None, :, :] == np.arange(N)[:, None, None]).astype(np.float32)


def rademacher(shape, seed: int = 0, purpose_extra: int = 0) -> np.ndarray:
    """Seeded +-1 direction (float32), e.g. for finite-difference probes."""
    return (_rng(seed, _S_DIR, purpose_extra).integers(0, 2, shape) * 2 - 1).astype(np.float32)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    """A synthetic segmentation problem: image recipe plus model parameters."""
    name: str
    W: int
    H: int
    N: int
    image_kind: str            # "disk" | "voronoi" | "voronoi_ramp" | "circles"
    sigma: float
    lam: float
    steps: int
    levels: int                # 0 = automatic coarsening
    tol: float
    pixel_units: bool = False  # h = 1 (eps = 2, tau = 4) instead of the unit square
    clip: bool = False
    ramp: float = 0.0
    n_regions: int = 0         # 0 -> N
    extra: dict = field(default_factory=dict)

    @property
    def h(self) -> float:
        return 1.0 if self.pixel_units else unit_spacing(self.W, self.H)

    @property
    def eps(self) -> float:
        return 2.0 * self.h

    @property
    def tau(self) -> float:
        return self.eps ** 2

    def scaled(self, W: int, H: Optional[int] = None, **kw) -> "Workload":
        """Same recipe on another lattice size (levels fall back to automatic)."""
        kw.setdefault("levels", 0)
        return replace(self, W=W, H=W if H is None else H, **kw)

    def make(self, seed: int = 0):
        """Return ``(image [C][H][W], u0 [N][H][W], labels [H][W])``, all seeded."""
        if self.image_kind == "disk":
            img, lab = disk_image(self.W, self.H, sigma=self.sigma, clip=self.clip, seed=seed)
        elif self.image_kind in ("voronoi", "voronoi_ramp"):
            img, lab = voronoi_image(self.W, self.H, self.n_regions or self.N, self.sigma,
                                     seed=seed, ramp=self.ramp, clip=self.clip)
        elif self.image_kind == "circles":
            img, lab = concentric_circles(self.W, self.H, seed=seed)
        else:
            raise ValueError(self.image_kind)
        u0 = random_simplex_field(self.N, self.H, self.W, seed=seed)
        return img, u0, lab


#: 64x64 disk, N = 2: the small case the oracle finishes in seconds
DISK64 = Workload("disk64_n2", 64, 64, 2, "disk", sigma=0.05, lam=50.0, steps=20,
                  levels=4, tol=1e-8, clip=True)
#: 1024x1024, 4 Voronoi regions, N = 4, 50 steps (headline throughput workload)
VORONOI1024 = Workload("voronoi1024_n4", 1024, 1024, 4, "voronoi", sigma=0.1, lam=100.0,
                       steps=50, levels=8, tol=1e-6)
#: 4096x4096, 8 Voronoi regions with linear ramps, N = 8, 30 steps (HBM-resident case)
VORONOI4096 = Workload("voronoi4096_n8", 4096, 4096, 8, "voronoi_ramp", sigma=0.1,
                       lam=100.0, steps=30, levels=10, tol=1e-6, ramp=0.2)
#: 512x512, N = 4, 20 steps: differentiation workload
VORONOI512 = Workload("voronoi512_n4", 512, 512, 4, "voronoi", sigma=0.1, lam=100.0,
                      steps=20, levels=0, tol=1e-6)

WORKLOADS = {w.name: w for w in (DISK64, VORONOI1024, VORONOI4096, VORONOI512)}


def pixel_twin(w: Workload, W: Optional[int] = None) -> Workload:
    """Same recipe on the pixel-unit scale (h = 1, eps = 2, tau = 4)."""
    kw = dict(name=w.name + "_px", pixel_units=True)
    if W is not None:
        kw.update(W=W, H=W, levels=0)
    return replace(w, **kw)


def batch_workloads(count: int = 256, seed: int = 0, min_side: int = 64, max_side: int = 1024,
                    n_choices=(2, 3, 4, 5, 6), sigma_range=(0.02, 0.15), steps: int = 30):
    """Heterogeneous batch: independent sides, phase counts and noise levels."""
    r = _rng(seed, _S_BATCH)
    out = []
    for b in range(count):
        W = int(r.integers(min_side, max_side + 1))
        H = int(r.integers(min_side, max_side + 1))
        N = int(r.choice(n_choices))
        s = float(r.uniform(*sigma_range))
        out.append(Workload(f"batch{b}", W, H, N, "voronoi", sigma=s, lam=100.0, steps=steps,
                            levels=0, tol=1e-6))
    return out
