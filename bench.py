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
# see profiles/k_cycle_voronoi1024_n4_batch8_traffic.md.  Must be re-measured
# whenever the kernel changes (absent: null).
TRAFFIC = {
    ("voronoi1024_n4", 8): 378.07e6,
    ("voronoi1024_n4", 1): 63.43e6,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def smoother_bytes_per_launch(N: int, C: int, n: int, sweeps: int, cycles: int, fixed: bool) -> float:
    """Algorithmic bytes of one k_cycle launch, averaged over a time step."""
    lpc = (sweeps + 1) // 2
    launches = cycles * lpc
    store_rhs = not (fixed and cycles == 1 and lpc == 1)
    first = 4 * (2 * N + C) + (4 * N if store_rhs else 0)
    later = 12 * N
    closing_means = 4 * C  # the image, for the colour-mean partials of a closing launch
    total = first + (launches - 1) * later + (cycles - 1 if not fixed else 0) * closing_means
    if launches > 1:
        total += closing_means
    return total * n / launches


def copy_calibration(mib: int, reps: int):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="segmentations timed")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="voronoi1024_n4")
    ap.add_argument("--batch", type=int, default=8,
                    help="images per batched solve (seeds 0..B-1, same shape); 1 = plain only")
    ap.add_argument("--schedule", choices=["fixed", "adaptive"], default="fixed",
                    help="fixed: every time step runs the cycle count found sufficient in a "
                         "calibration solve; adaptive: stop at the residual on the device")
    ap.add_argument("--cpu-sample-steps", type=int, default=6,
                    help="time steps of the oracle run for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB on the device (profiler counter calibration)")
    args = ap.parse_args()
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

    base = acseg.Problem.from_workload(w, C=C, levels=1, nu_pre=1, nu_post=1, max_cycles=20)

    # calibration: how many cycles does the slowest time step of any image need?
    cycles = 1
    for b in range(B):
        us[b].copy_(u0s[b])
        _, _, st, _ = acseg.solve(base, imgs[b], us[b])
        if st["status"] != acseg.OK:
            raise RuntimeError(f"calibration solve did not converge: {st}")
        cycles = max(cycles, st["cycles_max"])
    if args.schedule == "fixed":
        prob = acseg.Problem(**{**base.__dict__, "max_cycles": cycles,
                                "flags": acseg.FLAG_FIXED_CYCLES})
    else:
        prob = base
    log(f"[bench] {w.name}: {w.W}x{w.H} N={w.N} C={C} steps={w.steps} tol={w.tol} "
        f"schedule={args.schedule} cycles/step<={cycles} batch={B}")

    def segment():
        u.copy_(u0)
        _, c, _, _ = acseg.solve(prob, img, u, want_stats=False)
        return acseg.labels(prob, u, c)

    probs = [prob] * B

    def segment_batch():
        for b in range(B):
            us[b].copy_(u0s[b])
        _, cs, _ = acseg.solve_batched(probs, imgs, us, want_stats=False)
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
    if B > 1:
        elapsed = timed(segment_batch, args.steps)
        log(f"[bench] batched: {args.steps} x {B} segmentations in {elapsed:.4f} s")
    else:
        elapsed = elapsed_plain

    # the timed schedule converges: check it once with statistics
    u.copy_(u0)
    _, _, st_run, _ = acseg.solve(prob, img, u)
    if st_run["status"] != acseg.OK:
        raise RuntimeError(f"benchmark schedule did not converge: {st_run}")
    if B > 1:
        for b in range(B):
            us[b].copy_(u0s[b])
        _, _, sts = acseg.solve_batched(probs, imgs, us)
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
            w.N, C, n, prob.nu_pre + prob.nu_post,
            cycles if fixed else st_run["cycles_total"] / w.steps, fixed)
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": (int(TRAFFIC[(w.name, B)]) if (w.name, B) in TRAFFIC else None),
                "kernel": ("k_cycle_batch" if B > 1 else "k_cycle") +
                          " (time step: rhs + 2 red-black sweeps in LDS + residual + colour-mean partials)",
                "images_per_launch": B,
                "bytes_per_launch": int(bytes_per_launch), "avg_launch_us": round(avg_s * 1e6, 2),
                "launches": launches,
                "per_family_ms": {k: round(v[1] / reps, 4) for k, v in t.items()}}
        log(f"[bench] smoother {avg_s*1e6:.2f} us/launch -> {achieved:.1f} GB/s algorithmic")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as orc
        P = orc.Params.from_workload(w, C=C, tol=w.tol)
        k = args.cpu_sample_steps
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "batch": B, "W": w.W, "H": w.H, "N": w.N, "C": C,
                   "time_steps": w.steps, "lambda": w.lam, "h": w.h, "eps": w.eps, "tau": w.tau,
                   "tol": w.tol, "levels": prob.levels, "sweeps_per_cycle": prob.nu_pre + prob.nu_post,
                   "schedule": args.schedule, "cycles_per_step_max": cycles,
                   "cycles_total": st_run["cycles_total"], "final_residual": st_run["final_residual"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
