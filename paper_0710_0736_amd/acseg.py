"""Python binding of the gfx950 segmentation library (``include/acseg.h``).

Argument marshalling only: every step of the solve runs in the HIP kernels of
``libacseg.so``; torch provides device memory and the current stream.  There
is no CPU fallback -- if the library is missing or no GPU is present the calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, asdict, replace
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libacseg.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_NONFINITE = -2
ERR_WORKSPACE = -3
ERR_HIP = -4
ERR_UNSUPPORTED = -5
ERR_TOO_LARGE = -6
WARN_NOT_CONVERGED = 1
WARN_EMPTY_PHASE = 2
FLAG_STORE_CHECKPOINTS = 1
FLAG_FIXED_CYCLES = 2
FLAG_FIXED_C = 4
FLAG_NO_HOST_WAIT = 8
FLAG_SSC = 16
FLAG_REUSE_TABLES = 32
FLAG_SOR = 64


class _Problem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
                ("N", ctypes.c_int32), ("h", ctypes.c_double), ("eps", ctypes.c_double),
                ("lam", ctypes.c_double), ("tau", ctypes.c_double), ("steps", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("nu_pre", ctypes.c_int32),
                ("nu_post", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("steps_done", ctypes.c_int32),
                ("cycles_total", ctypes.c_int32), ("cycles_max", ctypes.c_int32),
                ("steps_not_converged", ctypes.c_int32), ("empty_phase_steps", ctypes.c_int32),
                ("final_residual", ctypes.c_double), ("max_residual", ctypes.c_double)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


@dataclass
class Problem:
    """Mirror of ``acseg_problem`` (see include/acseg.h for the meaning of each field)."""
    H: int
    W: int
    C: int
    N: int
    h: float
    eps: float
    lam: float
    tau: float
    steps: int = 0
    levels: int = 0
    nu_pre: int = 1
    nu_post: int = 1
    max_cycles: int = 50
    flags: int = 0
    tol: float = 1e-6

    def c(self) -> _Problem:
        d = asdict(self)
        return _Problem(*(d[k] for k, _ in _Problem._fields_))

    @classmethod
    def from_workload(cls, w, C: int = 3, **kw) -> "Problem":
        p = cls(H=w.H, W=w.W, C=C, N=w.N, h=w.h, eps=w.eps, lam=w.lam, tau=w.tau, steps=w.steps,
                levels=w.levels, tol=w.tol)
        return replace(p, **kw)


class AcsegError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


_lib = None
_ctx = {}
_ws_cache = {}


def lib():
    """Load libacseg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0710_0736_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        pp, sp = ctypes.POINTER(_Problem), ctypes.POINTER(_Stats)
        L.acseg_version.restype = ctypes.c_int32
        L.acseg_status_string.argtypes = [ctypes.c_int32]
        L.acseg_status_string.restype = ctypes.c_char_p
        L.acseg_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.acseg_destroy.argtypes = [vp]
        L.acseg_workspace_size.argtypes = [pp, ctypes.POINTER(sz)]
        L.acseg_project_simplex.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.acseg_transfer.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, vp, vp, vp]
        L.acseg_refine.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   vp, vp, vp]
        L.acseg_sample.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   vp, vp, vp]
        L.acseg_colour_space.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.acseg_mass_average.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.acseg_simplex_average.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.acseg_colour_means.argtypes = [vp, pp, vp, vp, vp, vp, sp, vp, sz, vp]
        L.acseg_step.argtypes = [vp, pp, vp, vp, vp, vp, vp, sp, vp, sz, vp]
        L.acseg_solve.argtypes = [vp, pp, vp, vp, vp, vp, sp, vp, sz, vp]
        L.acseg_solve_no_alloc.argtypes = [vp, pp, vp, vp, vp, vp, sp, vp]
        L.acseg_labels.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp]
        L.acseg_backward_workspace_size.argtypes = [pp, ctypes.POINTER(sz)]
        L.acseg_backward.argtypes = [vp, pp, vp, vp, vp, vp, vp, vp, vp, vp, sp, vp, sz, vp]
        L.acseg_batch_workspace_size.argtypes = [ctypes.c_int32, pp, ctypes.POINTER(sz)]
        L.acseg_solve_batched.argtypes = [vp, ctypes.c_int32, pp, ctypes.POINTER(vp),
                                          ctypes.POINTER(vp), ctypes.POINTER(vp), sp, vp, sz, vp]
        L.acseg_energy.argtypes = [vp, pp, vp, vp, vp, vp, sz, vp]
        L.acseg_timing_enable.argtypes = [vp, ctypes.c_int32]
        L.acseg_timing_read.argtypes = [vp, ctypes.POINTER(_KernelTime), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().acseg_status_string(code).decode()
    except Exception:
        return "status"


def _check(code: int, what: str):
    if code < 0:
        raise AcsegError(code, what)
    return code


def ctx(device: Optional[int] = None):
    if device is None:
        device = torch.cuda.current_device()
    if device not in _ctx:
        h = ctypes.c_void_p()
        _check(lib().acseg_create(device, ctypes.byref(h)), "acseg_create")
        _ctx[device] = h
    return _ctx[device]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, shape, dtype=torch.float32, name="tensor"):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def workspace_size(p: Problem) -> int:
    n = ctypes.c_size_t()
    _check(lib().acseg_workspace_size(ctypes.byref(p.c()), ctypes.byref(n)), "workspace_size")
    return n.value


def workspace(p: Problem, device=None) -> torch.Tensor:
    """A cached device workspace large enough for ``p`` (torch is the allocator)."""
    n = workspace_size(p)
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    ws = _ws_cache.get(dev)
    if ws is None or ws.numel() < n:
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        _ws_cache[dev] = ws
    return ws


def _stats_dict(s: _Stats) -> dict:
    return {k: getattr(s, k) for k, _ in _Stats._fields_}


# ---------------------------------------------------------------------------

def project_simplex(y: torch.Tensor) -> torch.Tensor:
    """Simplex projection of the columns of ``y`` ([N][count], float32, CUDA)."""
    N, count = y.shape
    _need(y, (N, count), name="y")
    x = torch.empty_like(y)
    _check(lib().acseg_project_simplex(ctx(y.device.index), N, count, _ptr(y), _ptr(x), _stream()),
           "acseg_project_simplex")
    return x


def prolong(vc: torch.Tensor, Wf: int, Hf: int) -> torch.Tensor:
    """P1 prolongation of [planes][ceil(Hf/2)][ceil(Wf/2)] onto the Wf x Hf lattice."""
    planes = vc.shape[0]
    _need(vc, (planes, (Hf + 1) // 2, (Wf + 1) // 2), name="vc")
    vf = torch.empty((planes, Hf, Wf), dtype=torch.float32, device=vc.device)
    _check(lib().acseg_transfer(ctx(vc.device.index), 0, planes, Wf, Hf, _ptr(vc), _ptr(vf),
                                _stream()), "acseg_transfer")
    return vf


def restrict(vf: torch.Tensor) -> torch.Tensor:
    """Transpose of ``prolong``: [planes][Hf][Wf] -> [planes][ceil(Hf/2)][ceil(Wf/2)]."""
    planes, Hf, Wf = vf.shape
    _need(vf, (planes, Hf, Wf), name="vf")
    vc = torch.empty((planes, (Hf + 1) // 2, (Wf + 1) // 2), dtype=torch.float32, device=vf.device)
    _check(lib().acseg_transfer(ctx(vf.device.index), 1, planes, Wf, Hf, _ptr(vf), _ptr(vc),
                                _stream()), "acseg_transfer")
    return vc


def refined_sides(W: int, H: int, r: int):
    """(Wf, Hf) of r uniform refinements of a W x H pixel lattice."""
    return ((W - 1) << r) + 1, ((H - 1) << r) + 1


def refine(src: torch.Tensor, r: int) -> torch.Tensor:
    """Piecewise-constant data on r refinements: [planes][H][W] -> [planes][Hf][Wf]."""
    planes, H, W = src.shape
    _need(src, (planes, H, W), name="src")
    Wf, Hf = refined_sides(W, H, r)
    dst = torch.empty((planes, Hf, Wf), dtype=torch.float32, device=src.device)
    _check(lib().acseg_refine(ctx(src.device.index), planes, W, H, r, _ptr(src), _ptr(dst), _stream()),
           "acseg_refine")
    return dst


def sample(src: torch.Tensor, W: int, H: int, r: int) -> torch.Tensor:
    """Values of a refined field at the pixel nodes: [planes][Hf][Wf] -> [planes][H][W]."""
    planes = src.shape[0]
    Wf, Hf = refined_sides(W, H, r)
    _need(src, (planes, Hf, Wf), name="src")
    dst = torch.empty((planes, H, W), dtype=torch.float32, device=src.device)
    _check(lib().acseg_sample(ctx(src.device.index), planes, W, H, r, _ptr(src), _ptr(dst), _stream()),
           "acseg_sample")
    return dst


def mass_average(img: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(M I) / m per channel: run the solver on it for consistent-mass fitting."""
    planes, H, W = img.shape
    _need(img, (planes, H, W), name="img")
    dst = torch.empty_like(img) if out is None else out
    _need(dst, (planes, H, W), name="out")
    _check(lib().acseg_mass_average(ctx(img.device.index), planes, W, H, _ptr(img), _ptr(dst), _stream()),
           "acseg_mass_average")
    return dst


def simplex_average(img: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The by-simplex view of the image (mean of the adjacent triangles' vertex
    means): run the solver on it for fitting with projection by simplex."""
    planes, H, W = img.shape
    _need(img, (planes, H, W), name="img")
    dst = torch.empty_like(img) if out is None else out
    _need(dst, (planes, H, W), name="out")
    _check(lib().acseg_simplex_average(ctx(img.device.index), planes, W, H, _ptr(img), _ptr(dst), _stream()),
           "acseg_simplex_average")
    return dst


LAB, AB = 0, 1


def colour_space(rgb: torch.Tensor, kind: int = LAB) -> torch.Tensor:
    """sRGB [3][...] in [0, 1] -> L*a*b* / 100 ([3][...]) or a*b* / 100 ([2][...])."""
    if rgb.shape[0] != 3:
        raise ValueError("rgb must have 3 channels")
    _need(rgb, tuple(rgb.shape), name="rgb")
    count = rgb[0].numel()
    dst = torch.empty((3 if kind == LAB else 2, *rgb.shape[1:]), dtype=torch.float32, device=rgb.device)
    _check(lib().acseg_colour_space(ctx(rgb.device.index), kind, count, _ptr(rgb), _ptr(dst), _stream()),
           "acseg_colour_space")
    return dst


def colour_means(p: Problem, image: torch.Tensor, u: torch.Tensor, c_prev=None):
    _need(image, (p.C, p.H, p.W), name="image")
    _need(u, (p.N, p.H, p.W), name="u")
    c = torch.empty((p.N, p.C), dtype=torch.float32, device=u.device)
    if c_prev is not None:
        _need(c_prev, (p.N, p.C), name="c_prev")
    ws = workspace(p, u.device.index)
    st = _Stats()
    _check(lib().acseg_colour_means(ctx(u.device.index), ctypes.byref(p.c()), _ptr(image), _ptr(u),
                                    _ptr(c_prev), _ptr(c), ctypes.byref(st), _ptr(ws), ws.numel(),
                                    _stream()), "acseg_colour_means")
    return c, _stats_dict(st)


def step(p: Problem, image: torch.Tensor, u_in: torch.Tensor, c_prev=None, want_stats=True,
         c_fixed=None):
    """One time step from ``u_in``; returns (u_out, c_used, stats).

    With ``c_fixed`` ([N][C]) the step uses those means (FLAG_FIXED_C)."""
    if c_fixed is not None:
        p = replace(p, flags=p.flags | FLAG_FIXED_C)
        c_prev = c_fixed
    _need(image, (p.C, p.H, p.W), name="image")
    _need(u_in, (p.N, p.H, p.W), name="u_in")
    if c_prev is not None:
        _need(c_prev, (p.N, p.C), name="c_prev")
    u_out = torch.empty_like(u_in)
    c = torch.empty((p.N, p.C), dtype=torch.float32, device=u_in.device)
    ws = workspace(p, u_in.device.index)
    st = _Stats()
    _check(lib().acseg_step(ctx(u_in.device.index), ctypes.byref(p.c()), _ptr(image), _ptr(u_in),
                            _ptr(u_out), _ptr(c_prev), _ptr(c),
                            ctypes.byref(st) if want_stats else None, _ptr(ws), ws.numel(),
                            _stream()), "acseg_step")
    return u_out, c, (_stats_dict(st) if want_stats else None)


def solve(p: Problem, image: torch.Tensor, u: torch.Tensor, checkpoints: bool = False,
          want_stats: bool = True, c_out: bool = True, c_fixed: Optional[torch.Tensor] = None):
    """``p.steps`` time steps; ``u`` (u^0) is overwritten with u^steps.

    Returns (u, c [N][C] of the result or None, stats or None, checkpoints or None).
    With ``c_fixed`` ([N][C]) every step uses those means (FLAG_FIXED_C) and c is c_fixed.
    """
    _need(image, (p.C, p.H, p.W), name="image")
    _need(u, (p.N, p.H, p.W), name="u")
    ck = None
    if checkpoints:
        p = replace(p, flags=p.flags | FLAG_STORE_CHECKPOINTS)
        ck = torch.empty((p.steps + 1, p.N, p.H, p.W), dtype=torch.float32, device=u.device)
    if c_fixed is not None:
        _need(c_fixed, (p.N, p.C), name="c_fixed")
        p = replace(p, flags=p.flags | FLAG_FIXED_C)
        c = c_fixed
    else:
        c = torch.empty((p.N, p.C), dtype=torch.float32, device=u.device) if c_out else None
    ws = workspace(p, u.device.index)
    st = _Stats()
    _check(lib().acseg_solve(ctx(u.device.index), ctypes.byref(p.c()), _ptr(image), _ptr(u),
                             _ptr(c), _ptr(ck), ctypes.byref(st) if want_stats else None,
                             _ptr(ws), ws.numel(), _stream()), "acseg_solve")
    return u, c, (_stats_dict(st) if want_stats else None), ck


def solve_no_alloc(p: Problem, image: torch.Tensor, u: torch.Tensor, c: Optional[torch.Tensor] = None,
                   checkpoints: Optional[torch.Tensor] = None, want_stats: bool = True):
    """``acseg_solve_no_alloc``: ``solve`` on the library's static scratch, with
    caller-owned outputs only (``u`` in/out, ``c`` [N][C] and ``checkpoints``
    [steps+1][N][H][W] when given), so the call itself allocates nothing.
    Returns the stats dict (or None)."""
    _need(image, (p.C, p.H, p.W), name="image")
    _need(u, (p.N, p.H, p.W), name="u")
    if c is not None:
        _need(c, (p.N, p.C), name="c")
    if checkpoints is not None:
        _need(checkpoints, (p.steps + 1, p.N, p.H, p.W), name="checkpoints")
        p = replace(p, flags=p.flags | FLAG_STORE_CHECKPOINTS)
    st = _Stats()
    _check(lib().acseg_solve_no_alloc(ctx(u.device.index), ctypes.byref(p.c()), _ptr(image), _ptr(u),
                                      _ptr(c), _ptr(checkpoints), ctypes.byref(st) if want_stats else None,
                                      _stream()), "acseg_solve_no_alloc")
    return _stats_dict(st) if want_stats else None


def _batch_arrays(problems):
    arr = (_Problem * len(problems))(*[p.c() for p in problems])
    return arr


def batch_workspace_size(problems) -> int:
    n = ctypes.c_size_t()
    _check(lib().acseg_batch_workspace_size(len(problems), _batch_arrays(problems), ctypes.byref(n)),
           "batch_workspace_size")
    return n.value


def solve_batched(problems, images, us, want_stats: bool = True, c_out: bool = True,
                  c_fixed=None, cs=None, reuse_tables: bool = False):
    """One time loop over independent images; every ``us[b]`` is overwritten.

    Returns (us, cs (list of [N][C] or None), stats (list) or None).  With
    ``c_fixed`` (a list of [N][C]) every step of image b uses c_fixed[b].
    ``cs`` (a list of [N][C]) receives the means instead of new tensors.  With
    ``reuse_tables`` the workspace keeps the descriptor tables of the previous
    call, which must have had the same problems, images, us and cs
    (FLAG_REUSE_TABLES); with a fixed schedule and ``want_stats=False`` the call
    can then be captured in a CUDA graph.
    """
    if c_fixed is not None:
        problems = [replace(p, flags=p.flags | FLAG_FIXED_C) for p in problems]
    if reuse_tables:
        problems = [replace(p, flags=p.flags | FLAG_REUSE_TABLES) for p in problems]
    B = len(problems)
    if not (len(images) == len(us) == B) or B == 0:
        raise ValueError("need one image and one field per problem")
    for p, im, u in zip(problems, images, us):
        _need(im, (p.C, p.H, p.W), name="image")
        _need(u, (p.N, p.H, p.W), name="u")
    dev = us[0].device
    if c_fixed is not None:
        cs = list(c_fixed)
        for p, c in zip(problems, cs):
            _need(c, (p.N, p.C), name="c_fixed")
        c_out = True
    elif cs is not None:
        for p, c in zip(problems, cs):
            _need(c, (p.N, p.C), name="cs")
        c_out = True
    else:
        cs = [torch.empty((p.N, p.C), dtype=torch.float32, device=dev) for p in problems] if c_out else None
    VP = ctypes.c_void_p * B
    ims = VP(*[im.data_ptr() for im in images])
    uus = VP(*[u.data_ptr() for u in us])
    ccs = VP(*[c.data_ptr() for c in cs]) if c_out else None
    n = batch_workspace_size(problems)
    ws = _ws_cache.get(("batch", dev))
    if ws is None or ws.numel() < n:
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        _ws_cache[("batch", dev)] = ws
    st = (_Stats * B)()
    _check(lib().acseg_solve_batched(ctx(dev.index), B, _batch_arrays(problems), ims, uus, ccs,
                                     st if want_stats else None, _ptr(ws), ws.numel(), _stream()),
           "acseg_solve_batched")
    return us, cs, ([_stats_dict(x) for x in st] if want_stats else None)


def backward(p: Problem, image: torch.Tensor, checkpoints: torch.Tensor, grad_uT: torch.Tensor,
             want_stats: bool = True, c_fixed: Optional[torch.Tensor] = None):
    """Gradients of L(u^steps) given dL/du^steps and the checkpoints of a solve.

    Returns (grad_image [C][H][W], grad_u0 [N][H][W], grad_params float64 [3]
    (lambda, eps at fixed tau, tau), grad_c [steps][N][C] -- or [N][C] =
    dL/dc_fixed for a solve with fixed means --, stats or None).
    """
    if c_fixed is not None:
        _need(c_fixed, (p.N, p.C), name="c_fixed")
        p = replace(p, flags=p.flags | FLAG_FIXED_C)
    _need(image, (p.C, p.H, p.W), name="image")
    _need(checkpoints, (p.steps + 1, p.N, p.H, p.W), name="checkpoints")
    _need(grad_uT, (p.N, p.H, p.W), name="grad_uT")
    dev = image.device
    gI = torch.empty_like(image)
    gu0 = torch.empty_like(grad_uT)
    gp = torch.empty(3, dtype=torch.float64, device=dev)
    gc = torch.empty((max(p.steps, 1), p.N, p.C), dtype=torch.float32, device=dev)
    n = ctypes.c_size_t()
    _check(lib().acseg_backward_workspace_size(ctypes.byref(p.c()), ctypes.byref(n)),
           "backward_workspace_size")
    ws = _ws_cache.get(("backward", dev))
    if ws is None or ws.numel() < n.value:
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
        _ws_cache[("backward", dev)] = ws
    st = _Stats()
    _check(lib().acseg_backward(ctx(dev.index), ctypes.byref(p.c()), _ptr(image), _ptr(checkpoints),
                                _ptr(c_fixed), _ptr(grad_uT), _ptr(gI), _ptr(gu0), _ptr(gp), _ptr(gc),
                                ctypes.byref(st) if want_stats else None, _ptr(ws), ws.numel(),
                                _stream()), "acseg_backward")
    gcv = gc[0] if c_fixed is not None else gc[:p.steps]
    return gI, gu0, gp, gcv, (_stats_dict(st) if want_stats else None)


class SegmentFn(torch.autograd.Function):
    """u^steps of a solve as a differentiable function of (image, u0, lambda, eps, tau).

    ``SegmentFn.apply(image, u0, lam, eps, tau, problem, c_fixed=None)``: lam,
    eps and tau are scalar tensors (they replace the problem's values); the
    gradient with respect to eps is taken at fixed tau.  With ``c_fixed``
    ([N][C]) every step uses those colour means, and they get a gradient too.
    The backward pass runs the library's adjoint from the checkpoints stored by
    the forward pass.
    """

    @staticmethod
    def forward(fctx, image, u0, lam, eps, tau, problem: Problem, c_fixed=None):
        p = replace(problem, lam=float(lam), eps=float(eps), tau=float(tau))
        img = image.detach().contiguous()
        u = u0.detach().clone().contiguous()
        cf = None if c_fixed is None else c_fixed.detach().float().contiguous()
        u, _, _, ck = solve(p, img, u, checkpoints=True, want_stats=False, c_out=False, c_fixed=cf)
        fctx.save_for_backward(img, ck)
        fctx.p = p
        fctx.cf = cf
        fctx.scalars = (lam, eps, tau)
        return u

    @staticmethod
    def backward(fctx, grad_u):
        img, ck = fctx.saved_tensors
        gI, gu0, gp, gc, _ = backward(fctx.p, img, ck, grad_u.contiguous().float(), want_stats=False,
                                      c_fixed=fctx.cf)
        outs = []
        for k, t in enumerate(fctx.scalars):
            outs.append(gp[k].to(t.device, t.dtype) if isinstance(t, torch.Tensor) else None)
        return (gI, gu0, *outs, None, gc if fctx.cf is not None else None)


def labels(p: Problem, u: torch.Tensor, c: torch.Tensor):
    """Returns (labels uint8 [H][W], composite [C][H][W], rounded composite [C][H][W])."""
    _need(u, (p.N, p.H, p.W), name="u")
    _need(c, (p.N, p.C), name="c")
    lab = torch.empty((p.H, p.W), dtype=torch.uint8, device=u.device)
    comp = torch.empty((p.C, p.H, p.W), dtype=torch.float32, device=u.device)
    rnd = torch.empty_like(comp)
    _check(lib().acseg_labels(ctx(u.device.index), ctypes.byref(p.c()), _ptr(u), _ptr(c), _ptr(lab),
                              _ptr(comp), _ptr(rnd), _stream()), "acseg_labels")
    return lab, comp, rnd


def energy(p: Problem, image: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """float64[4]: interface, concave, fitting, total (eq. E)."""
    _need(image, (p.C, p.H, p.W), name="image")
    _need(u, (p.N, p.H, p.W), name="u")
    e = torch.empty(4, dtype=torch.float64, device=u.device)
    ws = workspace(p, u.device.index)
    _check(lib().acseg_energy(ctx(u.device.index), ctypes.byref(p.c()), _ptr(image), _ptr(u),
                              _ptr(e), _ptr(ws), ws.numel(), _stream()), "acseg_energy")
    return e


def timing_enable(enable: bool = True, device=None):
    """Bracket the library's kernel launches with HIP events (profiling aid)."""
    _check(lib().acseg_timing_enable(ctx(device), 1 if enable else 0), "acseg_timing_enable")


def timing_read(device=None) -> dict:
    """{family: (launches, total_ms)} for the launches recorded since the last read."""
    buf = (_KernelTime * 16)()
    n = ctypes.c_int32()
    _check(lib().acseg_timing_read(ctx(device), buf, 16, ctypes.byref(n)), "acseg_timing_read")
    return {buf[k].name.decode(): (buf[k].launches, buf[k].total_ms) for k in range(n.value)}


def segment(image: torch.Tensor, N: int, *, lam: float, steps: int, h: Optional[float] = None,
            eps: Optional[float] = None, tau: Optional[float] = None, levels: int = 0,
            tol: float = 1e-6, u0: Optional[torch.Tensor] = None, seed: int = 0, **kw):
    """Segment a [C][H][W] float32 CUDA image into N phases.

    Defaults follow the unit-square scale: h = 1/(max(W, H) - 1), eps = 2h,
    tau = eps^2.  Returns (u, c, labels, stats).
    """
    C, H, W = image.shape
    h = 1.0 / (max(W, H) - 1) if h is None else h
    eps = 2.0 * h if eps is None else eps
    tau = eps * eps if tau is None else tau
    p = Problem(H=H, W=W, C=C, N=N, h=h, eps=eps, lam=lam, tau=tau, steps=steps, levels=levels,
                tol=tol, **kw)
    if u0 is None:
        from .synth import random_simplex_field
        u0 = torch.from_numpy(random_simplex_field(N, H, W, seed)).to(image.device)
    u = u0.clone().contiguous()
    u, c, st, _ = solve(p, image.contiguous(), u)
    lab, _, _ = labels(p, u, c)
    return u, c, lab, st


def segment_batch(images, Ns, *, lam: float, steps: int, tol: float = 1e-6, seed: int = 0, **kw):
    """Segment a list of [C][H][W] float32 CUDA images (phase counts ``Ns``, one
    per image or one for all) in one batched solve, at the unit-square scale of
    ``segment``.  Returns a list of (u, c, labels, stats)."""
    from .synth import random_simplex_field
    if isinstance(Ns, int):
        Ns = [Ns] * len(images)
    problems, us, ims = [], [], []
    for b, (image, N) in enumerate(zip(images, Ns)):
        C, H, W = image.shape
        h = 1.0 / (max(W, H) - 1)
        problems.append(Problem(H=H, W=W, C=C, N=N, h=h, eps=2.0 * h, lam=lam, tau=(2.0 * h) ** 2,
                                steps=steps, levels=1, tol=tol, **kw))
        us.append(torch.from_numpy(random_simplex_field(N, H, W, seed + b)).to(image.device))
        ims.append(image.contiguous())
    us, cs, sts = solve_batched(problems, ims, us)
    out = []
    for p, u, c, st in zip(problems, us, cs, sts):
        lab, _, _ = labels(p, u, c)
        out.append((u, c, lab, st))
    return out
