"""Host-side checks of the C ABI (no GPU needed).

* the built library loads and exports every function declared in include/acseg.h;
* host-side validation maps bad problems to the documented status codes
  (acseg_workspace_size validates without touching the device);
* the seeded workload generators are deterministic.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0710_0736_amd import acseg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "acseg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(acseg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = acseg.lib()
    names = declared_functions()
    assert "acseg_solve" in names and "acseg_step" in names
    for name in names:
        assert hasattr(L, name), name
    assert L.acseg_version() >= 100


def base_problem(**kw):
    p = acseg.Problem(H=64, W=48, C=3, N=4, h=1 / 63, eps=2 / 63, lam=100.0, tau=(2 / 63) ** 2,
                      steps=5, levels=1)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value,code", [
    ("N", 1, acseg.ERR_UNSUPPORTED), ("N", 9, acseg.ERR_UNSUPPORTED), ("C", 5, acseg.ERR_UNSUPPORTED),
    ("C", 0, acseg.ERR_INVALID_ARG), ("W", 1, acseg.ERR_INVALID_ARG), ("H", 0, acseg.ERR_INVALID_ARG),
    ("h", 0.0, acseg.ERR_INVALID_ARG), ("eps", -1.0, acseg.ERR_INVALID_ARG),
    ("tau", float("nan"), acseg.ERR_INVALID_ARG), ("lam", -0.5, acseg.ERR_INVALID_ARG),
    ("tol", -1e-6, acseg.ERR_INVALID_ARG), ("max_cycles", 0, acseg.ERR_INVALID_ARG),
    ("nu_pre", -1, acseg.ERR_INVALID_ARG), ("levels", 40, acseg.ERR_INVALID_ARG),
    ("flags", 1 << 20, acseg.ERR_INVALID_ARG),
])
def test_validation_codes(field, value, code):
    p = base_problem(**{field: value})
    n = ctypes.c_size_t()
    assert acseg.lib().acseg_workspace_size(ctypes.byref(p.c()), ctypes.byref(n)) == code


def test_workspace_size_grows_with_problem():
    a = acseg.workspace_size(base_problem())
    b = acseg.workspace_size(base_problem(W=96, H=128))
    assert 0 < a < b
    assert acseg.workspace_size(base_problem(nu_pre=0, nu_post=1)) == a


def test_status_strings():
    L = acseg.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, 1, 2):
        assert L.acseg_status_string(code).decode() not in ("", "unknown status")


def test_generators_are_deterministic():
    a = synth.VORONOI1024.scaled(96).make(3)
    b = synth.VORONOI1024.scaled(96).make(3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    img, u0, lab = a
    assert img.dtype == np.float32 and u0.dtype == np.float32
    assert np.abs(u0.sum(0) - 1).max() < 1e-6 and u0.min() > 0
    assert set(np.unique(lab)) <= set(range(4))


def _batch_code(problems):
    n = ctypes.c_size_t()
    arr = (acseg._Problem * max(1, len(problems)))(*[p.c() for p in problems])
    return acseg.lib().acseg_batch_workspace_size(len(problems), arr, ctypes.byref(n)), n.value


def test_batch_validation_codes():
    a, b = base_problem(), base_problem(W=96, H=33, N=3, C=1, lam=10.0)
    code, size = _batch_code([a, b])
    assert code == acseg.OK and size > acseg.workspace_size(a) + acseg.workspace_size(b)
    assert _batch_code([])[0] == acseg.ERR_INVALID_ARG
    assert _batch_code([a, base_problem(steps=6)])[0] == acseg.ERR_INVALID_ARG
    assert _batch_code([a, base_problem(max_cycles=7)])[0] == acseg.ERR_INVALID_ARG
    assert _batch_code([a, base_problem(nu_post=2)])[0] == acseg.ERR_INVALID_ARG
    ck = base_problem(flags=acseg.FLAG_STORE_CHECKPOINTS)
    assert _batch_code([ck])[0] == acseg.ERR_INVALID_ARG
    # multigrid images batch with Gauss-Seidel ones; the subspace correction does not batch
    assert _batch_code([a, base_problem(levels=2)])[0] == acseg.OK
    assert _batch_code([base_problem(levels=2, flags=acseg.FLAG_SSC)])[0] == acseg.ERR_UNSUPPORTED
    assert _batch_code([base_problem(levels=1, flags=acseg.FLAG_SSC)])[0] == acseg.OK
    assert _batch_code([a, base_problem(N=9)])[0] == acseg.ERR_UNSUPPORTED


def test_multigrid_validation_codes():
    n = ctypes.c_size_t()
    for kw, code in [(dict(levels=3, nu_pre=0, nu_post=2), acseg.ERR_UNSUPPORTED),
                     (dict(levels=3, nu_pre=2, nu_post=0), acseg.ERR_UNSUPPORTED),
                     (dict(levels=3), acseg.OK), (dict(levels=0), acseg.OK),
                     (dict(levels=1, nu_pre=0, nu_post=2), acseg.OK)]:
        p = base_problem(**kw)
        assert acseg.lib().acseg_workspace_size(ctypes.byref(p.c()), ctypes.byref(n)) == code, kw
    # the multigrid hierarchy needs its own buffers
    assert acseg.workspace_size(base_problem(levels=3)) > acseg.workspace_size(base_problem(levels=1))


def header_defines():
    text = open(os.path.join(ROOT, "include", "acseg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for name, val in re.findall(r"#define\s+ACSEG_(\w+)\s+\(?(-?\d+)u?\)?", text):
        out[name] = int(val)
    return out


def test_binding_constants_match_the_header():
    d = header_defines()
    flags = {k[len("FLAG_"):]: v for k, v in d.items() if k.startswith("FLAG_")}
    assert {"STORE_CHECKPOINTS", "FIXED_CYCLES", "FIXED_C", "NO_HOST_WAIT", "SSC", "REUSE_TABLES",
            "SOR"} <= set(flags)
    for name, v in flags.items():
        assert getattr(acseg, "FLAG_" + name) == v, name
    assert len(set(flags.values())) == len(flags)  # distinct bits
    for name in ("OK", "ERR_INVALID_ARG", "ERR_NONFINITE", "ERR_WORKSPACE", "ERR_HIP", "ERR_UNSUPPORTED",
                 "ERR_TOO_LARGE", "WARN_NOT_CONVERGED", "WARN_EMPTY_PHASE"):
        assert getattr(acseg, name) == d[name], name


def test_unknown_flag_bits_are_rejected():
    n = ctypes.c_size_t()
    for flags, ok in ((acseg.FLAG_SSC, True), (acseg.FLAG_REUSE_TABLES, True), (acseg.FLAG_SOR, True), (128, False),
                      (1 << 20, False)):
        p = base_problem(flags=flags)
        r = acseg.lib().acseg_workspace_size(ctypes.byref(p.c()), ctypes.byref(n))
        assert (r == acseg.OK) == ok, (flags, r)
