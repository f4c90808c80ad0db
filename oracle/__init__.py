"""FP64 CPU oracle for the vector-valued Allen-Cahn segmentation step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It wraps the plain C
library built from ``acseg_oracle.c`` (``python -m oracle.build``), which shares
no code with the HIP implementation.

Parity status: every function here is pinned by ``-m "not gpu"`` tests against
closed forms, textbook algorithms, library solvers or invariants (see
``tests/test_oracle_*.py``); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, asdict
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
                ("N", ctypes.c_int32), ("h", ctypes.c_double), ("eps", ctypes.c_double),
                ("lam", ctypes.c_double), ("tau", ctypes.c_double), ("levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("coarse_sweeps", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("ssc", ctypes.c_int32), ("tol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("empty_phase", ctypes.c_int32), ("nonmonotone", ctypes.c_int32),
                ("residual", ctypes.c_double), ("objective", ctypes.c_double)]


@dataclass
class Params:
    """Model and solver parameters (float64, unit conventions of the paper)."""
    H: int
    W: int
    C: int
    N: int
    h: float
    eps: float
    lam: float
    tau: float
    levels: int = 0          # 0 = automatic, 1 = Gauss-Seidel only
    nu_pre: int = 1
    nu_post: int = 1
    coarse_sweeps: int = 20
    max_cycles: int = 100000
    tol: float = 1e-10
    ssc: bool = False        # cycles = the paper's subspace correction over all basis functions

    def c(self) -> _Params:
        d = asdict(self)
        return _Params(d["H"], d["W"], d["C"], d["N"], d["h"], d["eps"], d["lam"], d["tau"],
                       d["levels"], d["nu_pre"], d["nu_post"], d["coarse_sweeps"],
                       d["max_cycles"], int(d["ssc"]), d["tol"])

    @classmethod
    def from_workload(cls, w, C: int = 3, **kw) -> "Params":
        p = cls(H=w.H, W=w.W, C=C, N=w.N, h=w.h, eps=w.eps, lam=w.lam, tau=w.tau,
                levels=w.levels)
        for k, v in kw.items():
            setattr(p, k, v)
        return p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        sp = ctypes.POINTER(_Stats)
        L.orc_project.argtypes = [ctypes.c_int, dp, dp]
        L.orc_auto_levels.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_prolong.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_restrict.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_colour_means.argtypes = [pp, dp, dp, dp, dp]
        L.orc_rhs.argtypes = [pp, dp, dp, dp, dp]
        L.orc_residual.argtypes = [pp, dp, dp]
        L.orc_residual.restype = ctypes.c_double
        L.orc_objective.argtypes = [pp, dp, dp]
        L.orc_objective.restype = ctypes.c_double
        L.orc_apply_H.argtypes = [pp, dp, dp]
        L.orc_solve_qp.argtypes = [pp, dp, dp, sp]
        L.orc_step.argtypes = [pp, dp, dp, dp, dp, dp, sp]
        L.orc_solve.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, sp]
        L.orc_energy.argtypes = [pp, dp, dp, dp, dp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_labels.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                 ctypes.POINTER(ctypes.c_uint8), dp, dp]
        L.orc_adjoint_solve.argtypes = [pp, dp, dp, dp]
        L.orc_adjoint_step.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_backward.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        L.orc_backward_c.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_solve_c.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, sp]
        L.orc_basis.argtypes = [pp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_ssc_update.argtypes = [pp, ctypes.c_int, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stats(s: _Stats) -> dict:
    return dict(cycles=s.cycles, converged=bool(s.converged), empty_phase=bool(s.empty_phase),
                nonmonotone=s.nonmonotone, residual=s.residual, objective=s.objective)


# ---------------------------------------------------------------------------

def project(y) -> tuple:
    """Projection of one vector onto the Gibbs simplex; returns (x, rounds)."""
    y = _d(y).ravel()
    x = np.empty_like(y)
    r = lib().orc_project(len(y), _p(y), _p(x))
    if r < 0:
        raise ValueError("bad N")
    return x, r


def auto_levels(W: int, H: int) -> int:
    return lib().orc_auto_levels(W, H)


def assemble(W: int, H: int, h: float):
    """Lumped mass [H][W] and stiffness stencils [H][W][3][3] (slot [dy+1][dx+1])."""
    m = np.empty((H, W))
    s = np.empty((H, W, 3, 3))
    lib().orc_assemble(W, H, h, _p(m), _p(s))
    return m, s


def prolong(vc: np.ndarray, Wf: int, Hf: int) -> np.ndarray:
    vc = _d(vc)
    N = vc.shape[0]
    vf = np.empty((N, Hf, Wf))
    lib().orc_prolong(Wf, Hf, N, _p(vc), _p(vf))
    return vf


def restrict(vf: np.ndarray) -> np.ndarray:
    vf = _d(vf)
    N, Hf, Wf = vf.shape
    vc = np.empty((N, (Hf + 1) // 2, (Wf + 1) // 2))
    lib().orc_restrict(Wf, Hf, N, _p(vf), _p(vc))
    return vc


def colour_means(P: Params, I, u, c_prev=None):
    """Returns (c [N][C], empty_flag)."""
    I, u = _d(I), _d(u)
    c = np.empty((P.N, P.C))
    cp = None if c_prev is None else _d(c_prev)
    e = lib().orc_colour_means(ctypes.byref(P.c()), _p(I), _p(u), _p(cp), _p(c))
    return c, bool(e)


def rhs(P: Params, I, un, c) -> np.ndarray:
    I, un, c = _d(I), _d(un), _d(c)
    b = np.empty((P.N, P.H, P.W))
    lib().orc_rhs(ctypes.byref(P.c()), _p(I), _p(un), _p(c), _p(b))
    return b


def residual(P: Params, b, u) -> float:
    return lib().orc_residual(ctypes.byref(P.c()), _p(_d(b)), _p(_d(u)))


def objective(P: Params, b, u) -> float:
    return lib().orc_objective(ctypes.byref(P.c()), _p(_d(b)), _p(_d(u)))


def apply_H(P: Params, v) -> np.ndarray:
    v = _d(v)
    out = np.empty_like(v)
    lib().orc_apply_H(ctypes.byref(P.c()), _p(v), _p(out))
    return out


def basis(P: Params, level: int, q: int) -> np.ndarray:
    """Basis function of node q (row-major) of ``level`` (0 = finest) on the
    finest lattice, [H][W] (Section "Multigrid Solution")."""
    eta = np.empty((P.H, P.W))
    if lib().orc_basis(ctypes.byref(P.c()), level, q, _p(eta)):
        raise ValueError("bad level or node")
    return eta


def ssc_update(P: Params, level: int, q: int, b, u):
    """One subspace correction of u along one basis function; returns
    (u_new, raised) where ``raised`` flags a rise of the step objective."""
    u = _d(u).copy()
    r = lib().orc_ssc_update(ctypes.byref(P.c()), level, q, _p(_d(b)), _p(u))
    if r < 0:
        raise ValueError("bad level or node")
    return u, bool(r)


def solve_qp(P: Params, b, u_init):
    u = _d(u_init).copy()
    st = _Stats()
    if lib().orc_solve_qp(ctypes.byref(P.c()), _p(_d(b)), _p(u), ctypes.byref(st)):
        raise ValueError("bad parameters")
    return u, _stats(st)


def step(P: Params, I, un, c_prev=None):
    """One time step; returns (u_next, c_used, stats)."""
    I, un = _d(I), _d(un)
    u = np.empty_like(un)
    c = np.empty((P.N, P.C))
    st = _Stats()
    cp = None if c_prev is None else _d(c_prev)
    if lib().orc_step(ctypes.byref(P.c()), _p(I), _p(un), _p(cp), _p(u), _p(c), ctypes.byref(st)):
        raise ValueError("bad parameters")
    return u, c, _stats(st)


def solve(P: Params, steps: int, I, u0, keep_trajectory: bool = True):
    """``steps`` time steps; returns (u_T, traj or None, c_traj [steps][N][C], stats list)."""
    I, u0 = _d(I), _d(u0)
    u = np.empty_like(u0)
    traj = np.empty((steps + 1,) + u0.shape) if keep_trajectory else None
    ct = np.empty((steps, P.N, P.C))
    st = (_Stats * max(steps, 1))()
    if lib().orc_solve(ctypes.byref(P.c()), steps, _p(I), _p(u0), _p(u), _p(traj), _p(ct), st):
        raise ValueError("bad parameters")
    return u, traj, ct, [_stats(st[k]) for k in range(steps)]


def energy(P: Params, I, u, c_prev=None):
    """Returns (total, [interface, concave, fitting])."""
    parts = np.empty(3)
    cp = None if c_prev is None else _d(c_prev)
    E = lib().orc_energy(ctypes.byref(P.c()), _p(_d(I)), _p(_d(u)), _p(cp), _p(parts))
    return E, parts


def labels(u, c):
    """Returns (labels uint8 [H][W], composite [C][H][W], rounded [C][H][W])."""
    u, c = _d(u), _d(c)
    N, H, W = u.shape
    C = c.shape[1]
    lab = np.empty((H, W), np.uint8)
    comp = np.empty((C, H, W))
    rnd = np.empty((C, H, W))
    lib().orc_labels(N, C, H, W, _p(u), _p(c), lab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                     _p(comp), _p(rnd))
    return lab, comp, rnd


def adjoint_solve(P: Params, unext, ubar):
    """z = (T H T)^+ T ubar with the free sets of unext (the gradient at b)."""
    unext, ubar = _d(unext), _d(ubar)
    z = np.empty_like(ubar)
    if lib().orc_adjoint_solve(ctypes.byref(P.c()), _p(unext), _p(ubar), _p(z)) < 0:
        raise ValueError("bad parameters")
    return z


def adjoint_step(P: Params, I, un, unext, ubar_next, c_prev=None):
    """One step backwards: returns (ubar_n, Ibar, grads [lambda, eps, tau], cbar [N][C])."""
    I, un, unext, ubar_next = _d(I), _d(un), _d(unext), _d(ubar_next)
    ubar_n = np.empty_like(un)
    Ibar = np.zeros_like(I)
    grads = np.zeros(3)
    cbar = np.empty((P.N, P.C))
    cp = None if c_prev is None else _d(c_prev)
    if lib().orc_adjoint_step(ctypes.byref(P.c()), _p(I), _p(un), _p(cp), _p(unext), _p(ubar_next),
                              _p(ubar_n), _p(Ibar), _p(grads), _p(cbar)):
        raise ValueError("bad parameters")
    return ubar_n, Ibar, grads, cbar


def backward(P: Params, steps: int, I, traj, ubar_T):
    """Backwards through a trajectory u^0..u^steps; returns (Ibar, grads, cbar, ubar0)."""
    I, traj, ubar_T = _d(I), _d(traj), _d(ubar_T)
    Ibar = np.empty_like(I)
    grads = np.empty(3)
    cbar = np.empty((max(steps, 1), P.N, P.C))
    ubar0 = np.empty_like(ubar_T)
    if lib().orc_backward(ctypes.byref(P.c()), steps, _p(I), _p(traj), _p(ubar_T), _p(Ibar),
                          _p(grads), _p(cbar), _p(ubar0)):
        raise ValueError("bad parameters")
    return Ibar, grads, cbar[:steps], ubar0


def solve_fixed_c(P: Params, steps: int, I, u0, c_fixed, keep_trajectory: bool = True):
    """``steps`` time steps with the colour means fixed; returns (u_T, traj or None, stats list)."""
    I, u0, cf = _d(I), _d(u0), _d(c_fixed)
    u = np.empty_like(u0)
    traj = np.empty((steps + 1,) + u0.shape) if keep_trajectory else None
    st = (_Stats * max(steps, 1))()
    if lib().orc_solve_c(ctypes.byref(P.c()), steps, _p(I), _p(u0), _p(cf), _p(u), _p(traj), st):
        raise ValueError("bad parameters")
    return u, traj, [_stats(st[k]) for k in range(steps)]


def backward_fixed_c(P: Params, steps: int, I, traj, c_fixed, ubar_T):
    """Backwards with fixed means; returns (Ibar, grads, cbar [N][C] = dL/dc_fixed, ubar0)."""
    I, traj, ubar_T, cf = _d(I), _d(traj), _d(ubar_T), _d(c_fixed)
    Ibar = np.empty_like(I)
    grads = np.empty(3)
    cbar = np.empty((P.N, P.C))
    ubar0 = np.empty_like(ubar_T)
    if lib().orc_backward_c(ctypes.byref(P.c()), steps, _p(I), _p(traj), _p(cf), _p(ubar_T), _p(Ibar),
                            _p(grads), _p(cbar), _p(ubar0)):
        raise ValueError("bad parameters")
    return Ibar, grads, cbar, ubar0
