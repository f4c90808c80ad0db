"""acseg_solve_no_alloc (the solve on the library's static scratch) against
acseg_solve on a caller workspace, through the C ABI.

The two share every kernel, so the results must agree bit for bit: the phase
fields, the colour means, the checkpoints and the statistics.  Two calls in a
row, the second on a smaller problem (the scratch keeps the first call's
contents, which the second must not read), and a problem beyond the scratch,
refused before anything runs.
"""
import numpy as np
import pytest
import torch

from paper_0710_0736_amd import acseg, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def run_both(w, seed, **kw):
    img, u0, _ = w.make(seed)
    p = acseg.Problem.from_workload(w, C=3, tol=1e-6, **kw)
    I, U0 = cuda(img), cuda(u0)
    u_ws, c_ws, st_ws, ck_ws = acseg.solve(p, I, U0.clone(), checkpoints=True)
    u_na = U0.clone()
    c_na = torch.empty((p.N, 3), dtype=torch.float32, device=DEV)
    ck_na = torch.empty_like(ck_ws)
    st_na = acseg.solve_no_alloc(p, I, u_na, c=c_na, checkpoints=ck_na)
    torch.cuda.synchronize()
    assert st_ws["status"] == acseg.OK, st_ws
    assert st_na == st_ws, (st_na, st_ws)
    assert torch.equal(u_na, u_ws)
    assert torch.equal(c_na, c_ws)
    assert torch.equal(ck_na, ck_ws)
    return st_na


def test_no_alloc_solve_equals_workspace_solve_twice():
    # first: the 1024^2 headline image with its 8-level hierarchy (about 65 of
    # the 80 MiB of scratch in use)
    big = synth.VORONOI1024.scaled(1024, steps=3)
    st = run_both(big, 1, levels=0, max_cycles=20)
    assert st["steps_done"] == 3
    # then a smaller lattice, another N, Gauss-Seidel cycles
    small = synth.VORONOI1024.scaled(77, 45, N=3, steps=4)
    st = run_both(small, 2, levels=1, max_cycles=50)
    assert st["steps_done"] == 4


def test_no_alloc_refuses_problems_beyond_its_scratch():
    w = synth.VORONOI4096.scaled(2048, 2048, steps=1)
    p = acseg.Problem.from_workload(w, C=3, levels=1)
    assert acseg.workspace_size(p) > 80 * 2 ** 20
    I = torch.zeros((3, p.H, p.W), dtype=torch.float32, device=DEV)
    u = torch.full((p.N, p.H, p.W), 1.0 / p.N, dtype=torch.float32, device=DEV)
    before = u.clone()
    with pytest.raises(acseg.AcsegError) as e:
        acseg.solve_no_alloc(p, I, u)
    assert e.value.code == acseg.ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert torch.equal(u, before)
