#!/usr/bin/env python3
"""Segmentation throughput on one MI355X.

One segmentation = all time steps of the vector-valued Allen-Cahn model on a
synthetic image (colour means, right-hand side, smoothing cycles to the
residual tolerance) plus the post-processing (colour means of the result,
labels, composite, rounded composite).  One benchmark step = one batched solve
of B such images (seeds 0..B-1, same shape; --batch, default 8); `value` is
segmentations per second, and `plain` gives the same images solved one per
call.  Inputs are resident in device memory before the timed region; only the
initial phase fields are restored (device copies) before every solve.

Default workload: 1024 x 1024 RGB, 4 Voronoi regions, noise sigma 0.1, N = 4
phases, eps = 2h, tau = eps^2, lambda = 100, 50 time steps, residual 1e-6.

The JSON line also carries
  roofline      the smoothing kernel's (k_cycle) algorithmic bytes per launch
                over its average launch time, measured with HIP events on the
                solve's stream.  A time step whose single launch builds the
                right-hand side, sweeps and closes the cycle reads u^n (4N B)
                and the image (4C B) and writes u^{n+1} (4N B) per node; a
                later launch reads u and the stored right-hand side and writes
                u (12N B per node);
  cpu_baseline  the FP64 oracle on one host core, timed on the first few time
                steps of the same workload and scaled to segmentations/s.

--copy-calibration runs only a plain device copy of a known size (for scaling
the DRAM byte counters of a profiler) and prints its size.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "segmentations/s at 1024² N=4 (batched vs plain); smoother GB/s vs HBM peak"
HBM_PEAK_GBS = 8000.0
# DRAM bytes per smoothing launch, (workload, images per launch) -> bytes:
# rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
# same counter reads for a 256 MiB device copy (FETCH x 2.000, WRITE x 1.000);
# see profiles/k_cycle_voronoi1024_n4_batch8_traffic.md and
# profiles/dram_per_kernel_hbm4096.md.  Measured on the fixed one-cycle
# schedule's launches only (keyed by workload, batch, cycles per step, levels,
# sweeps per cycle); must be re-measured whenever the kernel changes (absent:
# null).
TRAFFIC = {
    ("voronoi1024_n4", 8, 1, 1, 2): 374.67e6,
    ("voronoi1024_n4", 1, 1, 1, 2): 48.96e6,
    ("voronoi4096_n8", 1, 1, 1, 2): 1397.67e6,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def launches_per_cycle(levels: int, nu_pre: int, nu_post: int) -> int:
    """k_cycle launches per cycle: up to two sweeps per launch; a multigrid
    cycle smooths before and after its coarse correction in separate launches."""
    if levels == 1:
        return (nu_pre + nu_post + 1) // 2
    return (nu_pre + 1) // 2 + (nu_post + 1) // 2


def smoother_bytes_per_launch(N: int, C: int, n: int, lpc: int, cycles: int, fixed: bool) -> float:
    """Algorithmic bytes of one k_cycle launch, averaged over a time step."""
    launches = cycles * lpc
    store_rhs = not (fixed and cycles == 1 and lpc == 1)
    first = 4 * (2 * N + C) + (4 * N if store_rhs else 0)
    later = 12 * N
    closing_means = 4 * C  # the image, for the colour-mean partials of a closing launch
    total = first + (launches - 1) * later + (cycles - 1 if not fixed else 0) * closing_means
    if launches > 1:
        total += closing_means
    return total * n / launches


def sweep_bytes_per_launch(N: int, n: int, sweeps_per_cycle: int, lpc: int) -> float:
    """Sweep-equivalent bytes of one k_cycle launch: 12N bytes per node and sweep
    (read u and the right-hand side, write u, N float32 phases each) times the
    sweeps the launch performs."""
    return 12 * N * n * sweeps_per_cycle / lpc


def copy_calibration(mib: int, reps: int):
    """A plain device copy of a known size: bytes for counter calibration, and
    the copy's own bandwidth (read + written bytes / time) as the attainable
    streaming rate."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
                      "ms_per_copy": round(ms, 4), "GB_per_s": round(8 * n / ms / 1e6, 1)}), flush=True)


def run_hetero(args):
    """256 images of independent sizes and phase counts: one batched solve vs one call per image."""
    import torch
    from paper_0710_0736_amd import acseg, synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ws = synth.batch_workloads(args.hetero)
    made = [w.make(b) for b, w in enumerate(ws)]
    imgs = [torch.from_numpy(m[0]).to(dev) for m in made]
    u0s = [torch.from_numpy(m[1]).to(dev) for m in made]
    us = [torch.empty_like(u) for u in u0s]
    nodes = sum(w.W * w.H for w in ws)
    probs = [acseg.Problem.from_workload(w, C=3, levels=args.levels, max_cycles=args.max_cycles) for w in ws]
    cycles = 1
    for b in range(len(ws)):  # the slowest time step of any image fixes the schedule
        us[b].copy_(u0s[b])
        _, _, st, _ = acseg.solve(probs[b], imgs[b], us[b])
        if st["status"] != acseg.OK:
            raise RuntimeError(f"calibration solve of image {b} did not converge: {st}")
        cycles = max(cycles, st["cycles_max"])
    probs = [acseg.Problem(**{**p.__dict__, "max_cycles": cycles, "flags": acseg.FLAG_FIXED_CYCLES})
             for p in probs]

    def one_by_one():
        for b in range(len(ws)):
            us[b].copy_(u0s[b])
            acseg.solve(probs[b], imgs[b], us[b], want_stats=False, c_out=False)

    def batched():
        for b in range(len(ws)):
            us[b].copy_(u0s[b])
        acseg.solve_batched(probs, imgs, us, want_stats=False, c_out=False)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    k = max(1, args.steps // 4)
    t_plain = timed(one_by_one, k)
    t_batch = timed(batched, k)
    graph = None
    if not args.no_graph:
        # both forms captured in graphs: the batched solve reuses the tables an eager
        # call with the same arguments left in its workspace
        batched()
        torch.cuda.synchronize()
        ref = [x.clone() for x in us]
        gb = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gb):
            for b in range(len(ws)):
                us[b].copy_(u0s[b])
            acseg.solve_batched(probs, imgs, us, want_stats=False, c_out=False, reuse_tables=True)
        gp = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gp):
            one_by_one()
        t_gb = timed(gb.replay, k)
        same = all(torch.equal(x, y) for x, y in zip(us, ref))
        t_gp = timed(gp.replay, k)
        torch.cuda.synchronize()
        same = same and all(torch.equal(x, y) for x, y in zip(us, ref))
        if not same:
            raise RuntimeError("graph replays differ from the eager solves")
        graph = {"batched": round(len(ws) / t_gb, 2), "plain": round(len(ws) / t_gp, 2), "unit": "images/s",
                 "replay_equals_eager": same}
        log(f"[bench] hetero graphs: batched {len(ws) / t_gb:.1f} images/s, one call per image {len(ws) / t_gp:.1f}")
    for b in range(len(ws)):
        us[b].copy_(u0s[b])
    _, _, sts = acseg.solve_batched(probs, imgs, us)
    bad = [x for x in sts if x["status"] != acseg.OK]
    if bad:
        raise RuntimeError(f"batched schedule did not converge: {bad[0]}")
    roof, groups = None, None
    if not args.no_roofline:
        lpc = launches_per_cycle(probs[0].levels, probs[0].nu_pre, probs[0].nu_post)
        spc = probs[0].nu_pre + probs[0].nu_post
        steps = ws[0].steps

        def family_times(members):
            acseg.timing_enable(True)
            acseg.timing_read()
            for b in members:
                us[b].copy_(u0s[b])
            acseg.solve_batched([probs[b] for b in members], [imgs[b] for b in members],
                                [us[b] for b in members], want_stats=False, c_out=False)
            torch.cuda.synchronize()
            t = acseg.timing_read()
            acseg.timing_enable(False)
            return t

        def smoother_rates(members, t):
            launches, ms = t["smooth"]
            sweep = sum(sweep_bytes_per_launch(ws[b].N, ws[b].W * ws[b].H, spc, lpc) for b in members)
            comp = sum(smoother_bytes_per_launch(ws[b].N, 3, ws[b].W * ws[b].H, lpc, cycles, True)
                       for b in members)
            per_step = cycles * lpc * steps  # launches of one image's solve
            total_s = ms / 1e3
            return launches, total_s, sweep * per_step / total_s / 1e9, comp * per_step / total_s / 1e9

        everyone = list(range(len(ws)))
        t_all = family_times(everyone)
        launches, total_s, sweep_gbs, comp_gbs = smoother_rates(everyone, t_all)
        roof = {"bound": "hbm", "achieved": round(sweep_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(sweep_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_cycle_batch (one launch per (N, C) group and smoothing launch)",
                "avg_launch_us": round(total_s / launches * 1e6, 2), "launches": launches,
                "compulsory": {"achieved": round(comp_gbs, 1), "frac": round(comp_gbs / HBM_PEAK_GBS, 4)},
                "per_family_ms": {k: round(v[1], 4) for k, v in t_all.items()},
                "per_family_avg_launch_us": {k: round(v[1] / v[0] * 1e3, 2) for k, v in t_all.items()}}
        # each (N, C) group alone: its launch time and rate show what a launch's
        # tail costs when fewer tiles share it
        groups = []
        for N in sorted({w.N for w in ws}):
            members = [b for b in everyone if ws[b].N == N]
            t_g = family_times(members)
            gl, gs, g_sweep, g_comp = smoother_rates(members, t_g)
            tiles = sum(((ws[b].W + 63) // 64) * ((ws[b].H + (31 if N <= 3 else 15)) // (32 if N <= 3 else 16))
                        for b in members)
            groups.append({"N": N, "images": len(members), "nodes": sum(ws[b].W * ws[b].H for b in members),
                           "tiles_per_launch": tiles, "tiles_per_cu": round(tiles / 256, 1),
                           "avg_launch_us": round(gs / gl * 1e6, 2), "achieved": round(g_sweep, 1),
                           "frac": round(g_sweep / HBM_PEAK_GBS, 4),
                           "compulsory_frac": round(g_comp / HBM_PEAK_GBS, 4)})
        # a launch merged over every group would move all bytes at the best group's
        # rate at most: the time that would save bounds what merging can gain
        best = max(g["achieved"] for g in groups)
        merged_s = sweep_gbs * total_s / best
        roof["merge_gain_bound_frac"] = round(1 - merged_s / total_s, 4)
        log(f"[bench] hetero smoother: {sweep_gbs:.1f} GB/s sweep-equivalent over {launches} launches; "
            f"groups: " + ", ".join(f"N={g['N']} {g['avg_launch_us']} us {g['achieved']} GB/s" for g in groups))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as orc
        rng = np.random.default_rng(2024)
        sample = sorted(rng.choice(len(ws), size=min(8, len(ws)), replace=False).tolist())
        k = args.cpu_sample_steps or 2
        tc = 0.0
        for b in sample:
            P = orc.Params.from_workload(ws[b], C=3, tol=ws[b].tol)
            t0c = time.perf_counter()
            orc.solve(P, k, made[b][0], made[b][1], keep_trajectory=False)
            tc += time.perf_counter() - t0c
        work_sample = sum(ws[b].W * ws[b].H * ws[b].N * k for b in sample)
        work_all = sum(w.W * w.H * w.N * w.steps for w in ws)
        t_all_cpu = tc * work_all / work_sample
        cpu = {"value": round(len(ws) / t_all_cpu, 6), "unit": "images/s", "cores": 1, "kind": "oracle",
               "sample": f"first {k} of {ws[0].steps} time steps of 8 images drawn from the batch "
                         f"(indices {sample}), FP64, single thread, {tc:.1f} s; extrapolated to the whole "
                         f"batch by node-phase count (W H N x time steps)"}
        log(f"[bench] oracle: {tc:.2f} s for {k} time steps of 8 sampled images")

    out = {"metric": "images/s, heterogeneous batch (batched vs one call per image)",
           "value": round(len(ws) / t_batch, 2), "unit": "images/s", "n_gpus": 1, "steps": k,
           "warmup": 1, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "plain": {"value": round(len(ws) / t_plain, 2), "unit": "images/s",
                     "ms_per_batch": round(t_plain * 1e3, 3)},
           "graph": graph,
           "config": {"workload": f"hetero{len(ws)}", "images": len(ws), "nodes": nodes,
                      "N": sorted({w.N for w in ws}), "time_steps": ws[0].steps,
                      "cycles_per_step": cycles, "sweeps_per_cycle": 2, "levels": probs[0].levels},
           "roofline": roof, "groups": groups, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_refined(args):
    """Segmentation on a refined lattice: pixel data refined r times by
    piecewise-constant injection, the solve on the refined lattice, the phase
    fields sampled back at the pixels and labelled there."""
    import torch
    from paper_0710_0736_amd import acseg, synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    r, Wp, N, C, steps = args.refine, args.refine_pixels, 4, 3, 50
    Wf, Hf = acseg.refined_sides(Wp, Wp, r)
    img_np, _ = synth.voronoi_image(Wp, Wp, N, 0.1, seed=0, channels=C)
    Ip = torch.from_numpy(img_np).to(dev)
    U0 = torch.from_numpy(synth.random_simplex_field(N, Hf, Wf, seed=0)).to(dev)
    u = torch.empty_like(U0)
    h = 1.0 / (1 << r)   # the pixel is the unit of length
    eps = 0.5            # half a pixel: 2^(r-1) refined nodes
    base = acseg.Problem(H=Hf, W=Wf, C=C, N=N, h=h, eps=eps, lam=100.0, tau=eps * eps, steps=steps,
                         levels=args.levels, tol=1e-6, nu_pre=args.nu[0], nu_post=args.nu[1],
                         max_cycles=args.max_cycles, flags=acseg.FLAG_SOR if args.sor else 0)
    pix = acseg.Problem(H=Wp, W=Wp, C=C, N=N, h=1.0, eps=eps, lam=100.0, tau=eps * eps, steps=steps)
    If = acseg.refine(Ip, r)
    u.copy_(U0)
    _, _, st, _ = acseg.solve(base, If, u)
    if st["status"] != acseg.OK:
        raise RuntimeError(f"calibration solve did not converge: {st}")
    cycles = max(1, st["cycles_max"])
    prob = acseg.Problem(**{**base.__dict__, "max_cycles": cycles, "flags": acseg.FLAG_FIXED_CYCLES | base.flags})
    log(f"[bench] refined: {Wp}^2 pixels, r={r} -> {Wf}x{Hf} nodes, levels={prob.levels}, "
        f"cycles/step<={cycles}")

    def segment():
        Ifine = acseg.refine(Ip, r)
        u.copy_(U0)
        _, c, _, _ = acseg.solve(prob, Ifine, u, want_stats=False)
        return acseg.labels(pix, acseg.sample(u, Wp, Wp, r), c)

    for _ in range(args.warmup):
        segment()
    torch.cuda.synchronize()
    k = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(k):
        segment()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / k
    u.copy_(U0)
    _, _, st_run, _ = acseg.solve(prob, If, u)
    if st_run["status"] != acseg.OK:
        raise RuntimeError(f"benchmark schedule did not converge: {st_run}")
    acseg.timing_enable(True)
    acseg.timing_read()
    segment()
    torch.cuda.synchronize()
    tm = acseg.timing_read()
    acseg.timing_enable(False)
    launches, total_ms = tm["smooth"]
    avg_s = total_ms / launches / 1e3
    lpc = launches_per_cycle(prob.levels, prob.nu_pre, prob.nu_post)
    bpl = smoother_bytes_per_launch(N, C, Wf * Hf, lpc, cycles, True)
    achieved = bpl / avg_s / 1e9
    spl = sweep_bytes_per_launch(N, Wf * Hf, prob.nu_pre + prob.nu_post, lpc)
    sweep_achieved = spl / avg_s / 1e9
    out = {"metric": "segmentations/s on a refined lattice (refine + solve + sample + labels)",
           "value": round(1.0 / t, 3), "unit": "segmentations/s", "n_gpus": 1, "steps": k,
           "warmup": args.warmup, "ms_per_step": round(t * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"voronoi{Wp}_n{N}_refined{r}" + ("_sor" if args.sor else ""), "pixels": Wp * Wp, "r": r, "W": Wf, "H": Hf,
                      "N": N, "C": C, "h": h, "eps": eps, "tau": eps * eps, "lambda": 100.0,
                      "time_steps": steps, "levels": prob.levels,
                      "sweeps_per_cycle": prob.nu_pre + prob.nu_post, "cycles_per_step_max": cycles,
                      "cycles_total": st_run["cycles_total"], "final_residual": st_run["final_residual"]},
           "roofline": {"bound": "hbm", "achieved": round(sweep_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(sweep_achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_cycle",
                        "bytes_per_launch": int(spl), "avg_launch_us": round(avg_s * 1e6, 2),
                        "compulsory": {"bytes_per_launch": int(bpl), "achieved": round(achieved, 1),
                                       "frac": round(achieved / HBM_PEAK_GBS, 4)},
                        "launches": launches,
                        "per_family_ms": {kk: round(v[1], 4) for kk, v in tm.items()}},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Forward solve with checkpoints, then gradients of a squared-error loss."""
    import torch
    from paper_0710_0736_amd import acseg, synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.WORKLOADS["voronoi512_n4"]
    if args.pixel_units:
        w = synth.pixel_twin(w)
    img_np, u0_np, lab = w.make(0)
    I = torch.from_numpy(img_np).to(dev)
    U0 = torch.from_numpy(u0_np).to(dev)
    y = torch.from_numpy(np.stack([(lab == i) for i in range(w.N)]).astype(np.float32)).to(dev)
    p = acseg.Problem.from_workload(w, C=3, levels=args.levels, max_cycles=args.max_cycles,
                                    flags=(acseg.FLAG_SSC if args.ssc else 0) | (acseg.FLAG_SOR if args.sor else 0))
    st = {}

    def forward():
        u, _, s, ck = acseg.solve(p, I, U0.clone(), checkpoints=True, want_stats=False, c_out=False)
        return u, ck

    def both():
        u, ck = forward()
        return acseg.backward(p, I, ck, 2 * (u - y), want_stats=False)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    k = max(2, args.steps)
    t_f = timed(forward, k)
    t_fb = timed(both, k)
    u, ck = forward()
    _, _, _, _, bst = acseg.backward(p, I, ck, 2 * (u - y))
    _, _, fst, _ = acseg.solve(p, I, U0.clone())
    gbar = 2 * (u - y)
    roof = None
    if not args.no_roofline:
        acseg.timing_enable(True)
        acseg.timing_read()
        reps = 3
        for _ in range(reps):
            acseg.backward(p, I, ck, gbar, want_stats=False)
        torch.cuda.synchronize()
        tm = acseg.timing_read()
        acseg.timing_enable(False)
        launches, ms = tm["adj_sweep"]
        n = w.W * w.H
        # 12N bytes per node and sweep (read z and the loss gradient, write z);
        # the launch also reads the free sets, 16N per node per launch compulsory
        sweep_bytes = 12 * w.N * n * bst["cycles_total"] * reps
        comp_bytes = 16 * w.N * n * launches
        sec = ms / 1e3
        roof = {"bound": "hbm", "achieved": round(sweep_bytes / sec / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(sweep_bytes / sec / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_adj_sweep (two red-black sweeps of the adjoint solve per launch)",
                "sweeps_per_backward": bst["cycles_total"], "launches_per_backward": launches // reps,
                "avg_launch_us": round(ms / launches * 1e3, 2),
                "compulsory": {"achieved": round(comp_bytes / sec / 1e9, 1),
                               "frac": round(comp_bytes / sec / 1e9 / HBM_PEAK_GBS, 4)},
                "per_family_ms": {kk: round(v[1] / reps, 4) for kk, v in tm.items()},
                "per_family_launches": {kk: v[0] // reps for kk, v in tm.items()}}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as orc
        P = orc.Params.from_workload(w, C=3, tol=w.tol)
        t0c = time.perf_counter()
        uT, traj, _, _ = orc.solve(P, w.steps, img_np, u0_np)
        t1c = time.perf_counter()
        orc.backward(P, w.steps, img_np, traj, 2 * (uT - y.cpu().numpy().astype(np.float64)))
        t2c = time.perf_counter()
        cpu = {"value": round((t2c - t0c) * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"the whole workload: {w.steps} FP64 time steps forward ({(t1c - t0c):.1f} s, "
                         f"levels={P.levels}, tol={P.tol}) and the adjoint through all of them "
                         f"({(t2c - t1c):.1f} s), single thread",
               "backward_ms": round((t2c - t1c) * 1e3, 1)}
        log(f"[bench] oracle: forward {t1c - t0c:.2f} s, backward {t2c - t1c:.2f} s")
    out = {"metric": f"adjoint: forward+backward time per segmentation ({w.name}{'_sor' if args.sor else ''})",
           "value": round(t_fb * 1e3, 3), "unit": "ms", "n_gpus": 1, "steps": k, "warmup": 1,
           "ms_per_step": round(t_fb * 1e3, 3), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "forward_ms": round(t_f * 1e3, 3), "backward_ms": round((t_fb - t_f) * 1e3, 3),
           "backward_over_forward": round((t_fb - t_f) / t_f, 2),
           "config": {"workload": w.name, "W": w.W, "H": w.H, "N": w.N, "time_steps": w.steps,
                      "levels": p.levels, "forward_cycles_total": fst["cycles_total"],
                      "forward_cycles_max": fst["cycles_max"], "forward_status": fst["status"],
                      "adjoint_sweeps_total": bst["cycles_total"], "adjoint_sweeps_max": bst["cycles_max"],
                      "status": bst["status"]},
           "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="segmentations timed")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="voronoi1024_n4")
    ap.add_argument("--pixel-units", action="store_true",
                    help="the workload's pixel-unit twin (h = 1, eps = 2, tau = 4)")
    ap.add_argument("--levels", type=int, default=1,
                    help="multigrid levels (1: Gauss-Seidel cycles only, 0: automatic)")
    ap.add_argument("--max-cycles", type=int, default=20, help="cycle budget per time step")
    ap.add_argument("--cycles", type=int, default=0,
                    help="fixed cycles per time step without a calibration solve (0: calibrate)")
    ap.add_argument("--nu", type=int, nargs=2, default=(1, 1), metavar=("PRE", "POST"),
                    help="smoothing sweeps before / after the coarse correction")
    ap.add_argument("--vcycle-levels", type=int, default=-1,
                    help="levels of the V-cycle solve timed beside a Gauss-Seidel bench line "
                         "(-1: the workload's configured hierarchy; 0: none)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the batched segmentation eagerly only (default: also as a captured graph, "
                         "which gives `value`)")
    ap.add_argument("--sor", action="store_true",
                    help="over-relaxed smoothing sweeps (ACSEG_FLAG_SOR)")
    ap.add_argument("--ssc", action="store_true",
                    help="coarse correction = the paper's subspace correction over all basis functions")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time a forward solve with checkpoints and the backward pass "
                         "(voronoi512_n4: 512^2, N = 4, 20 steps)")
    ap.add_argument("--batch", type=int, default=8,
                    help="images per batched solve (seeds 0..B-1, same shape); 1 = plain only")
    ap.add_argument("--schedule", choices=["fixed", "adaptive"], default="fixed",
                    help="fixed: every time step runs the cycle count found sufficient in a "
                         "calibration solve; adaptive: stop at the residual on the device")
    ap.add_argument("--cpu-sample-steps", type=int, default=0,
                    help="time steps of the oracle run for the CPU baseline (0: about 6 steps of "
                         "a 1024^2 N=4 image's work, at least 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB on the device (profiler counter calibration)")
    ap.add_argument("--hetero", type=int, default=0, metavar="B",
                    help="only time a batch of B images of independent sizes (64..1024) and "
                         "phase counts (2..6), batched vs one call per image")
    ap.add_argument("--refine", type=int, default=0, metavar="R",
                    help="only time segmentation on R uniform refinements of a pixel image "
                         "(--refine-pixels square, N = 4, eps half a pixel)")
    ap.add_argument("--refine-pixels", type=int, default=128)
    ap.add_argument("--simplex-projection", action="store_true",
                    help="fitting with projection by simplex (the by-simplex view of each image, per segmentation)")
    ap.add_argument("--consistent-mass", action="store_true",
                    help="fitting with the consistent mass matrix (the solver runs on M I / m)")
    args = ap.parse_args()
    if args.refine:
        run_refined(args)
        return
    if args.hetero:
        if args.levels != 1:
            # a 256-image run with multigrid cycles ended in a host segmentation
            # fault whose cause has not been found: refused until it is
            sys.exit("bench.py --hetero runs Gauss-Seidel cycles only (--levels 1); "
                     "the multigrid form is disabled until a crash it showed is explained")
        run_hetero(args)
        return
    if args.adjoint:
        run_adjoint(args)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(1, args.steps))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0710_0736_amd import acseg, synth

    w = synth.WORKLOADS[args.workload]
    if args.pixel_units:
        w = synth.pixel_twin(w)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = max(1, args.batch)
    made = [w.make(seed) for seed in range(B)]
    img_np, u0_np, _ = made[0]
    C = img_np.shape[0]
    n = w.W * w.H
    imgs = [torch.from_numpy(m[0]).to(dev) for m in made]
    u0s = [torch.from_numpy(m[1]).to(dev) for m in made]
    us = [torch.empty_like(u0) for u0 in u0s]
    img, u0, u = imgs[0], u0s[0], us[0]

    ssc_flag = (acseg.FLAG_SSC if args.ssc else 0) | (acseg.FLAG_SOR if args.sor else 0)
    # a workload's tolerance below 1e-6 is the FP64 oracle's; the FP32 solve stops at 1e-6,
    # above its rounding floor of about 1e-7
    gpu_tol = max(w.tol, 1e-6)
    base = acseg.Problem.from_workload(w, C=C, levels=args.levels, nu_pre=args.nu[0],
                                       nu_post=args.nu[1], max_cycles=args.max_cycles, flags=ssc_flag,
                                       tol=gpu_tol)

    # consistent-mass fitting: the solver runs on M I / m, computed per segmentation
    # into a fixed buffer per image
    avg = {id(x): torch.empty_like(x) for x in imgs}
    if args.consistent_mass:
        prep = lambda x: acseg.mass_average(x, out=avg[id(x)])  # noqa: E731
    elif args.simplex_projection:
        prep = lambda x: acseg.simplex_average(x, out=avg[id(x)])  # noqa: E731
    else:
        prep = lambda x: x  # noqa: E731
    # calibration: how many cycles does the slowest time step of any image need?
    cycles = max(1, args.cycles)
    for b in (range(B) if args.cycles == 0 else ()):
        us[b].copy_(u0s[b])
        _, _, st, _ = acseg.solve(base, prep(imgs[b]), us[b])
        if st["status"] != acseg.OK:
            raise RuntimeError(f"calibration solve did not converge: {st}")
        cycles = max(cycles, st["cycles_max"])
    if args.schedule == "fixed":
        prob = acseg.Problem(**{**base.__dict__, "max_cycles": cycles,
                                "flags": acseg.FLAG_FIXED_CYCLES | ssc_flag})
    else:
        prob = base
    log(f"[bench] {w.name}: {w.W}x{w.H} N={w.N} C={C} steps={w.steps} tol={gpu_tol} "
        f"schedule={args.schedule} cycles/step<={cycles} batch={B}")

    def segment():
        u.copy_(u0)
        _, c, _, _ = acseg.solve(prob, prep(img), u, want_stats=False)
        return acseg.labels(prob, u, c)

    probs = [prob] * B

    def segment_batch():
        ims = [prep(x) for x in imgs]
        for b in range(B):
            us[b].copy_(u0s[b])
        _, cs, _ = acseg.solve_batched(probs, ims, us, want_stats=False)
        return [acseg.labels(prob, us[b], cs[b]) for b in range(B)]

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    elapsed_plain = timed(segment, args.steps)
    log(f"[bench] plain: {args.steps} segmentations in {elapsed_plain:.4f} s")
    elapsed_eager = None
    graph_info = None
    if B > 1:
        elapsed = elapsed_eager = timed(segment_batch, args.steps)
        log(f"[bench] batched: {args.steps} x {B} segmentations in {elapsed:.4f} s")
        if not args.no_graph:
            # one batched segmentation (restore u^0, solve, labels) captured in a graph
            # and replayed: the solve reuses the descriptor tables that an eager call
            # with the same arguments left in its workspace, so it enqueues kernels only
            cs_g = [torch.empty((w.N, C), dtype=torch.float32, device=dev) for _ in range(B)]
            ims_g = [prep(x) for x in imgs]
            for b in range(B):
                us[b].copy_(u0s[b])
            acseg.solve_batched(probs, ims_g, us, want_stats=False, cs=cs_g)  # uploads the tables
            ref = [x.clone() for x in us]
            torch.cuda.synchronize()

            def body():
                ims = [prep(x) for x in imgs]
                for b in range(B):
                    us[b].copy_(u0s[b])
                acseg.solve_batched(probs, ims, us, want_stats=False, cs=cs_g, reuse_tables=True)
                return [acseg.labels(prob, us[b], cs_g[b]) for b in range(B)]

            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                body()
            elapsed_graph = timed(g.replay, args.steps)
            torch.cuda.synchronize()
            same = all(torch.equal(us[b], ref[b]) for b in range(B))
            if not same:
                raise RuntimeError("graph replay of the batched segmentation differs from the eager solve")
            log(f"[bench] batched, graph replay: {args.steps} x {B} segmentations in {elapsed_graph:.4f} s")
            graph_info = {"replay_equals_eager": same}
            elapsed = elapsed_graph
    else:
        elapsed = elapsed_plain

    # the configuration's own hierarchy (config text: 8-level V-cycles), one image per
    # call, timed beside the headline: same converged steps, a coarse correction per cycle
    vcycle = None
    vlevels = w.levels if args.vcycle_levels < 0 else args.vcycle_levels
    if vlevels > 1 and prob.levels == 1 and not args.pixel_units:
        pv = acseg.Problem(**{**base.__dict__, "levels": vlevels, "max_cycles": args.max_cycles})
        u.copy_(u0)
        _, _, stv, _ = acseg.solve(pv, prep(img), u)
        if stv["status"] != acseg.OK:
            raise RuntimeError(f"V-cycle calibration did not converge: {stv}")
        pvf = acseg.Problem(**{**pv.__dict__, "max_cycles": stv["cycles_max"],
                               "flags": acseg.FLAG_FIXED_CYCLES | ssc_flag})

        def segment_v():
            u.copy_(u0)
            _, c, _, _ = acseg.solve(pvf, prep(img), u, want_stats=False)
            return acseg.labels(pvf, u, c)

        tv = timed(segment_v, args.steps)
        u.copy_(u0)
        _, _, stv2, _ = acseg.solve(pvf, prep(img), u)
        if stv2["status"] != acseg.OK:
            raise RuntimeError(f"V-cycle schedule did not converge: {stv2}")
        # the same cycle budget with exits on the device: a step's cycles after its
        # residual meets the tolerance do nothing, and the host never waits
        pvd = acseg.Problem(**{**pv.__dict__, "max_cycles": stv["cycles_max"],
                               "flags": acseg.FLAG_NO_HOST_WAIT | ssc_flag})

        def segment_vd():
            u.copy_(u0)
            _, c, _, _ = acseg.solve(pvd, prep(img), u, want_stats=False)
            return acseg.labels(pvd, u, c)

        tvd = timed(segment_vd, args.steps)
        u.copy_(u0)
        _, _, stv3, _ = acseg.solve(pvd, prep(img), u)
        if stv3["status"] != acseg.OK:
            raise RuntimeError(f"V-cycle schedule with device exits did not converge: {stv3}")
        vcycle = {"levels": vlevels, "value": round(args.steps / tvd, 3), "unit": "segmentations/s",
                  "ms_per_segmentation": round(tvd / args.steps * 1e3, 4), "batch": 1,
                  "schedule": "device exits (at most cycles_per_step_max cycles; the converged ones do nothing)",
                  "cycles_total": stv3["cycles_total"], "cycles_per_step_max": stv["cycles_max"],
                  "final_residual": stv3["final_residual"],
                  "fixed_schedule": {"value": round(args.steps / tv, 3), "unit": "segmentations/s",
                                     "cycles_total": stv2["cycles_total"],
                                     "final_residual": stv2["final_residual"]}}
        log(f"[bench] {vlevels}-level V-cycles, one image per call: {args.steps} segmentations in "
            f"{tvd:.4f} s with device exits ({stv3['cycles_total']} cycles), {tv:.4f} s fixed")
        if B > 1:
            # the same V-cycles over the headline's batch (eager, device exits)
            probs_v = [pvd] * B

            def segment_vb():
                ims = [prep(x) for x in imgs]
                for b in range(B):
                    us[b].copy_(u0s[b])
                _, cs, _ = acseg.solve_batched(probs_v, ims, us, want_stats=False)
                return [acseg.labels(pvd, us[b], cs[b]) for b in range(B)]

            tvb = timed(segment_vb, args.steps)
            for b in range(B):
                us[b].copy_(u0s[b])
            _, _, stsb = acseg.solve_batched(probs_v, [prep(x) for x in imgs], us)
            if any(x["status"] != acseg.OK for x in stsb):
                raise RuntimeError(f"batched V-cycles did not converge: {stsb}")
            vcycle["batched"] = {"value": round(args.steps * B / tvb, 3), "unit": "segmentations/s",
                                 "batch": B, "graph": False,
                                 "cycles_total": [x["cycles_total"] for x in stsb],
                                 "final_residual_max": max(x["final_residual"] for x in stsb)}
            log(f"[bench] {vlevels}-level V-cycles, batched: {args.steps} x {B} segmentations in {tvb:.4f} s")

    # the timed schedule converges: check it once with statistics
    u.copy_(u0)
    _, _, st_run, _ = acseg.solve(prob, prep(img), u)
    if st_run["status"] != acseg.OK:
        raise RuntimeError(f"benchmark schedule did not converge: {st_run}")
    if B > 1:
        for b in range(B):
            us[b].copy_(u0s[b])
        _, _, sts = acseg.solve_batched(probs, [prep(x) for x in imgs], us)
        bad = [x for x in sts if x["status"] != acseg.OK]
        if bad:
            raise RuntimeError(f"batched schedule did not converge: {bad[0]}")

    roof = None
    if not args.no_roofline:
        acseg.timing_enable(True)
        acseg.timing_read()
        reps = max(2, min(args.steps, 10))
        for _ in range(reps):
            segment_batch() if B > 1 else segment()
        torch.cuda.synchronize()
        t = acseg.timing_read()
        acseg.timing_enable(False)
        launches, total_ms = t["smooth"]
        avg_s = total_ms / launches / 1e3
        fixed = args.schedule == "fixed"
        bytes_per_launch = B * smoother_bytes_per_launch(
            w.N, C, n, launches_per_cycle(prob.levels, prob.nu_pre, prob.nu_post),
            cycles if fixed else st_run["cycles_total"] / w.steps, fixed)
        achieved = bytes_per_launch / avg_s / 1e9
        lpc = launches_per_cycle(prob.levels, prob.nu_pre, prob.nu_post)
        sweep_bytes = B * sweep_bytes_per_launch(w.N, n, prob.nu_pre + prob.nu_post, lpc)
        sweep_achieved = sweep_bytes / avg_s / 1e9
        tkey = (w.name + ("_consistent_mass" if args.consistent_mass else "")
                + ("_simplex_projection" if args.simplex_projection else ""), B, cycles, prob.levels,
                prob.nu_pre + prob.nu_post)
        # `achieved`/`frac`: the sweep-equivalent bytes (12N per node and sweep); the
        # LDS temporal blocking keeps most of them out of HBM, so `compulsory` gives
        # the bytes a launch cannot avoid (read u and I, write u) over the same time
        roof = {"bound": "hbm", "achieved": round(sweep_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(sweep_achieved / HBM_PEAK_GBS, 4),
                "traffic": (int(TRAFFIC[tkey]) if fixed and tkey in TRAFFIC else None),
                "kernel": ("k_cycle_batch" if B > 1 else "k_cycle") +
                          " (time step: rhs + 2 red-black sweeps in LDS + residual + colour-mean partials)",
                "images_per_launch": B, "sweeps_per_launch": (prob.nu_pre + prob.nu_post) / lpc,
                "bytes_per_launch": int(sweep_bytes), "avg_launch_us": round(avg_s * 1e6, 2),
                "compulsory": {"bytes_per_launch": int(bytes_per_launch), "achieved": round(achieved, 1),
                               "frac": round(achieved / HBM_PEAK_GBS, 4)},
                "launches": launches,
                "per_family_ms": {k: round(v[1] / reps, 4) for k, v in t.items()}}
        # the attainable streaming rate for the same bytes: a plain device copy that
        # reads and writes half of them each
        ncp = max(1, int(bytes_per_launch) // 8)
        src_cp = torch.ones(ncp, dtype=torch.float32, device=dev)
        dst_cp = torch.empty_like(src_cp)
        dst_cp.copy_(src_cp)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(20):
            dst_cp.copy_(src_cp)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 8 * ncp / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9
        del src_cp, dst_cp
        roof["compulsory"]["copy_same_bytes_GBs"] = round(copy_gbs, 1)
        roof["compulsory"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
        log(f"[bench] smoother {avg_s*1e6:.2f} us/launch -> {sweep_achieved:.1f} GB/s sweep-equivalent, "
            f"{achieved:.1f} GB/s compulsory (a device copy of the compulsory bytes: {copy_gbs:.1f} GB/s)")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as orc
        P = orc.Params.from_workload(w, C=C, tol=w.tol)
        k = args.cpu_sample_steps or max(1, min(w.steps, round(6 * (1024 * 1024 * 4) / (n * w.N))))
        t0c = time.perf_counter()
        orc.solve(P, k, img_np, u0_np, keep_trajectory=False)
        tc = time.perf_counter() - t0c
        per_seg = tc / k * w.steps
        cpu = {"value": round(1.0 / per_seg, 6), "unit": "segmentations/s", "cores": 1,
               "kind": "oracle",
               "sample": f"first {k} of {w.steps} time steps of the same image, FP64, levels="
                         f"{P.levels}, tol={P.tol}, single thread; scaled by {w.steps}/{k}"}
        log(f"[bench] oracle: {tc:.2f} s for {k} time steps")

    out = {
        "metric": METRIC,
        "value": round(B * args.steps / elapsed, 3),
        "unit": "segmentations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "plain": {"value": round(args.steps / elapsed_plain, 3), "unit": "segmentations/s",
                  "ms_per_segmentation": round(elapsed_plain / args.steps * 1e3, 4)},
        "batched_eager": (None if elapsed_eager is None else
                          {"value": round(B * args.steps / elapsed_eager, 3), "unit": "segmentations/s"}),
        "graph": graph_info,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name + ("_consistent_mass" if args.consistent_mass else "")
                               + ("_simplex_projection" if args.simplex_projection else "")
                               + ("_ssc" if args.ssc and prob.levels != 1 else "") + ("_sor" if args.sor else ""),
                   "batch": B,
                   "W": w.W, "H": w.H, "N": w.N, "C": C,
                   "time_steps": w.steps, "lambda": w.lam, "h": w.h, "eps": w.eps, "tau": w.tau,
                   "tol": gpu_tol, "levels": prob.levels, "sweeps_per_cycle": prob.nu_pre + prob.nu_post,
                   "coarse_correction": ("subspace correction" if args.ssc else "truncated") if prob.levels != 1 else None,
                   "schedule": args.schedule, "cycles_per_step_max": cycles,
                   "cycles_total": st_run["cycles_total"], "final_residual": st_run["final_residual"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "vcycle": vcycle,
    }
    # absolute smoothing rate: full-image red-black sweeps of the finest lattice per
    # second (and the node updates they make)
    sweeps = B * args.steps * st_run["cycles_total"] * (prob.nu_pre + prob.nu_post) / elapsed
    out["sweeps_per_s"] = round(sweeps, 1)
    out["node_sweeps_per_s"] = round(sweeps * n, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
