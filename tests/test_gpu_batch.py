"""The batched solve against one-image solves.

Every image of a batch runs the same kernels on the same tiles with its own
convergence control, and every reduction has a fixed order, so each result
must be bit-identical to the one-image solve of the same problem.  The
one-image solve itself is held to the oracle by test_gpu_parity.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from paper_0710_0736_amd import acseg, synth
from test_gpu_parity import cuda

pytestmark = pytest.mark.gpu

SPECS = [  # W, H, N, C, lambda, seed
    (96, 80, 4, 3, 100.0, 1), (37, 53, 3, 3, 50.0, 2), (150, 64, 2, 1, 100.0, 3),
    (64, 64, 4, 3, 20.0, 4), (200, 120, 3, 3, 100.0, 5), (70, 130, 4, 3, 100.0, 6),
]


def make_batch(pixel: bool, steps: int, max_cycles: int, flags: int = 0):
    problems, images, u0s = [], [], []
    for (W, H, N, C, lam, seed) in SPECS:
        base = synth.pixel_twin(synth.VORONOI1024) if pixel else synth.VORONOI1024
        w = base.scaled(W, H, N=N, lam=lam)
        img, u0, _ = w.make(seed)
        if C == 1:
            img = img.mean(axis=0, keepdims=True)
        problems.append(acseg.Problem.from_workload(w, C=C, levels=1, steps=steps, tol=1e-6,
                                                    max_cycles=max_cycles, flags=flags))
        images.append(cuda(img))
        u0s.append(cuda(u0))
    return problems, images, u0s


@pytest.mark.parametrize("pixel,fixed", [(False, False), (False, True), (True, False)])
def test_batched_equals_single(pixel, fixed):
    steps = 3 if pixel else 6
    flags = acseg.FLAG_FIXED_CYCLES if fixed else 0
    problems, images, u0s = make_batch(pixel, steps, 4 if fixed else 300, flags)
    singles = []
    for p, im, u0 in zip(problems, images, u0s):
        u, c, st, _ = acseg.solve(p, im, u0.clone())
        singles.append((u, c, st))
    us = [u0.clone() for u0 in u0s]
    us, cs, sts = acseg.solve_batched(problems, images, us)
    torch.cuda.synchronize()
    for b, (u, c, st) in enumerate(singles):
        assert torch.equal(us[b], u), b
        assert torch.equal(cs[b], c), b
        assert sts[b] == st, (b, sts[b], st)
    if pixel:  # the images converge after different cycle counts
        assert len({st["cycles_total"] for _, _, st in singles}) > 1


def test_bench_configuration_eight_full_size_images():
    """The launch shape of the benchmark: 8 full-size headline images (seeds
    0..7) in one batched solve on the fixed one-cycle schedule, each
    bit-identical to its single-image solve (whose parity with the oracle is
    tested at full size)."""
    w = synth.VORONOI1024
    p = acseg.Problem.from_workload(w, levels=1, steps=3, max_cycles=1, flags=acseg.FLAG_FIXED_CYCLES)
    made = [w.make(s) for s in range(8)]
    images = [cuda(m[0]) for m in made]
    u0s = [cuda(m[1]) for m in made]
    us, cs, sts = acseg.solve_batched([p] * 8, images, [u.clone() for u in u0s])
    torch.cuda.synchronize()
    for b in range(8):
        u, c, st, _ = acseg.solve(p, images[b], u0s[b].clone())
        assert torch.equal(us[b], u) and torch.equal(cs[b], c), b
        assert sts[b]["status"] == acseg.OK and sts[b] == st, (b, sts[b], st)


def test_batch_of_one_full_size_image_and_repeat_calls():
    w = synth.VORONOI1024
    img, u0, _ = w.make(0)
    p = acseg.Problem.from_workload(w, levels=1, steps=4, max_cycles=1, flags=acseg.FLAG_FIXED_CYCLES)
    I, U0 = cuda(img), cuda(u0)
    u_s, c_s, st_s, _ = acseg.solve(p, I, U0.clone())
    for _ in range(2):  # the descriptor upload of one call must not disturb the next
        us, cs, sts = acseg.solve_batched([p, p], [I, I], [U0.clone(), U0.clone()])
        torch.cuda.synchronize()
        for b in range(2):
            assert torch.equal(us[b], u_s) and torch.equal(cs[b], c_s)
            assert sts[b]["final_residual"] == st_s["final_residual"]


def test_segment_and_segment_batch_agree():
    ims = []
    for (W, H, N, seed) in [(80, 64, 3, 11), (50, 70, 4, 12)]:
        w = synth.VORONOI1024.scaled(W, H, N=N)
        img, _, _ = w.make(seed)
        ims.append((cuda(img), N))
    res = acseg.segment_batch([im for im, _ in ims], [N for _, N in ims], lam=100.0, steps=5, seed=3)
    for b, (im, N) in enumerate(ims):
        u, c, lab, st = acseg.segment(im, N, lam=100.0, steps=5, seed=3 + b, levels=1)
        torch.cuda.synchronize()
        assert st["status"] == acseg.OK and res[b][3]["status"] == acseg.OK
        assert torch.equal(res[b][0], u) and torch.equal(res[b][2], lab)


def config5_sample(count=10, seed=11):
    """A sample of the heterogeneous-batch workload at reduced sides: independent
    sides in [64, 200], noise sigma in [0.02, 0.15], Voronoi regions = N, every
    phase count 2..6 twice (N = 5 and 6 have kernels of their own), RGB, unit
    scale, 30 time steps."""
    ws = synth.batch_workloads(count, seed=seed, min_side=64, max_side=200)
    return [replace(w, N=2 + b % 5) for b, w in enumerate(ws)]


def test_batched_against_oracle_config5_sample():
    """Each image of a batched solve against the oracle: the final field of 30
    steps against the oracle's trajectory (max |du| <= 1e-4 and the label
    gate), and single steps taken by batched solves from the oracle's own
    states (rounded to float32) at the start, middle and end."""
    from test_gpu_parity import GATE_U, host, label_gate
    import oracle as orc
    ws = config5_sample()
    assert sorted({w.N for w in ws}) == [2, 3, 4, 5, 6]
    made = [w.make(b) for b, w in enumerate(ws)]
    refs = []
    for w, (img, u0, _) in zip(ws, made):
        P = orc.Params.from_workload(w, C=3, tol=1e-11, levels=1)
        _, traj, ct, sts = orc.solve(P, w.steps, img, u0)
        assert all(s["converged"] for s in sts)
        refs.append((P, traj, ct))
    probs = [acseg.Problem.from_workload(w, C=3, levels=1, tol=1e-6, max_cycles=60) for w in ws]
    us, cs, sts = acseg.solve_batched(probs, [cuda(m[0]) for m in made], [cuda(m[1]) for m in made])
    torch.cuda.synchronize()
    for b, (w, (P, traj, ct)) in enumerate(zip(ws, refs)):
        assert sts[b]["status"] == acseg.OK and sts[b]["steps_done"] == w.steps, (b, sts[b])
        ug = host(us[b])
        err = np.abs(ug - traj[-1]).max()
        assert err <= GATE_U, (b, w.N, w.W, w.H, err)
        bad, total, raw = label_gate(ug, traj[-1])
        assert bad <= 1e-3 * total, (b, bad, raw)
    # per step, from the oracle's states: one batched call per step index
    one = [acseg.Problem(**{**p.__dict__, "steps": 1}) for p in probs]
    for n in (0, 15, 29):
        starts = [np.asarray(traj[n], np.float32) for (_, traj, _) in refs]
        us, cs, sts = acseg.solve_batched(one, [cuda(m[0]) for m in made], [cuda(s) for s in starts])
        torch.cuda.synchronize()
        for b, (w, (P, traj, ct)) in enumerate(zip(ws, refs)):
            u_ref, c_ref, st_ref = orc.step(P, made[b][0], starts[b], ct[n - 1] if n > 0 else None)
            assert st_ref["converged"]
            assert np.abs(host(cs[b]) - orc.colour_means(P, made[b][0], u_ref, c_ref)[0]).max() < 1e-5
            ug = host(us[b])
            assert sts[b]["status"] == acseg.OK and sts[b]["final_residual"] <= 1e-6, (n, b, sts[b])
            err = np.abs(ug - u_ref).max()
            assert err <= GATE_U, (n, b, w.N, err)
            bad, total, raw = label_gate(ug, u_ref)
            assert bad <= 1e-3 * total, (n, b, bad, raw)


MG_SPECS = [  # W, H, N, C, lambda, seed, levels: tails from level 1 and 2, and none (levels = 2)
    (96, 80, 4, 3, 100.0, 1, 0), (37, 53, 3, 3, 50.0, 2, 0), (150, 64, 2, 1, 100.0, 3, 0),
    (200, 120, 5, 3, 100.0, 5, 0), (70, 130, 6, 3, 100.0, 6, 0), (160, 140, 4, 3, 100.0, 7, 2),
]


def make_mg_batch(pixel: bool, steps: int, max_cycles: int, flags: int = 0):
    problems, images, u0s = [], [], []
    for (W, H, N, C, lam, seed, levels) in MG_SPECS:
        base = synth.pixel_twin(synth.VORONOI1024) if pixel else synth.VORONOI1024
        w = base.scaled(W, H, N=N, lam=lam)
        img, u0, _ = w.make(seed)
        if C == 1:
            img = img.mean(axis=0, keepdims=True)
        problems.append(acseg.Problem.from_workload(w, C=C, levels=levels, steps=steps, tol=1e-6,
                                                    max_cycles=max_cycles, flags=flags))
        images.append(cuda(img))
        u0s.append(cuda(u0))
    return problems, images, u0s


@pytest.mark.parametrize("pixel,fixed,sor", [(True, False, False), (True, True, False), (False, False, False),
                                             (True, False, True)])
def test_batched_multigrid_equals_single(pixel, fixed, sor):
    """Multigrid cycles over a batch (one launch per pass over the images that
    have the pass's level: images with an LDS tail from level 1 or 2 and one
    whose coarsest level is a global pass) give each image exactly its
    one-image solve."""
    steps = 3
    flags = (acseg.FLAG_FIXED_CYCLES if fixed else 0) | (acseg.FLAG_SOR if sor else 0)
    problems, images, u0s = make_mg_batch(pixel, steps, 6 if fixed else 200, flags)
    singles = []
    for p, im, u0 in zip(problems, images, u0s):
        u, c, st, _ = acseg.solve(p, im, u0.clone())
        singles.append((u, c, st))
    us = [u0.clone() for u0 in u0s]
    us, cs, sts = acseg.solve_batched(problems, images, us)
    torch.cuda.synchronize()
    for b, (u, c, st) in enumerate(singles):
        assert torch.equal(us[b], u), b
        assert torch.equal(cs[b], c), b
        assert sts[b] == st, (b, sts[b], st)
        if not fixed:
            assert st["status"] == acseg.OK, (b, st)


def test_batched_multigrid_step_against_oracle():
    """One batched multigrid step of every image in pixel units against the
    oracle's step (the per-step gates of the one-image tests)."""
    from test_gpu_parity import GATE_U, host, label_gate
    import oracle as orc
    problems, images, u0s = make_mg_batch(True, 1, 200)
    us, cs, sts = acseg.solve_batched(problems, images, [u.clone() for u in u0s])
    torch.cuda.synchronize()
    for b, (W, H, N, C, lam, seed, levels) in enumerate(MG_SPECS):
        w = synth.pixel_twin(synth.VORONOI1024).scaled(W, H, N=N, lam=lam)
        img = images[b].cpu().numpy().astype(np.float64)
        P = orc.Params.from_workload(w, C=C, tol=1e-12, levels=0)
        u_ref, c_ref, st_ref = orc.step(P, img, host(u0s[b]))
        assert st_ref["converged"]
        assert sts[b]["status"] == acseg.OK and sts[b]["final_residual"] <= 1e-6, (b, sts[b])
        ug = host(us[b])
        err = np.abs(ug - u_ref).max()
        assert err <= GATE_U, (b, err)
        bad, total, raw = label_gate(ug, u_ref)
        assert bad <= 1e-3 * total, (b, bad, raw)


def test_multigrid_passes_equal_across_workgroup_sizes():
    """A down or up pass runs 1024, 512 or 256 threads per workgroup, the most
    that let all of its workgroups be resident at once, so a batch and a single
    image of the same size take different variants (on a 256-CU device: six
    512^2 images put 1536 workgroups into the level-1 up pass and 768 into the
    level-1 down pass, against 256 and 128 for one image).  Every node is
    updated by the same arithmetic whichever thread takes it, so the batch
    must give each image exactly its one-image solve."""
    base = synth.pixel_twin(synth.VORONOI1024)
    problems, images, u0s = [], [], []
    for seed in range(6):
        w = base.scaled(512, 512, N=4)
        img, u0, _ = w.make(20 + seed)
        problems.append(acseg.Problem.from_workload(w, levels=0, steps=2, max_cycles=3,
                                                    flags=acseg.FLAG_FIXED_CYCLES))
        images.append(cuda(img))
        u0s.append(cuda(u0))
    singles = [acseg.solve(p, im, u0.clone())[:3] for p, im, u0 in zip(problems, images, u0s)]
    us, cs, sts = acseg.solve_batched(problems, images, [u0.clone() for u0 in u0s])
    torch.cuda.synchronize()
    for b, (u, c, st) in enumerate(singles):
        assert torch.equal(us[b], u), b
        assert torch.equal(cs[b], c), b
        assert sts[b] == st, (b, sts[b], st)
