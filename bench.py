#!/usr/bin/env python3
"""Segmentation throughput on one MI355X.

One benchmark step = one complete segmentation of a synthetic image: all time
steps of the vector-valued Allen-Cahn model (colour means, right-hand side,
smoothing cycles to the residual tolerance) plus the post-processing (colour
means of the result, labels, composite, rounded composite).  Inputs are
resident in device memory before the timed region; only the initial phase
field is restored (a device copy) before every segmentation.

Default workload: 1024 x 1024 RGB, 4 Voronoi regions, noise sigma 0.1, N = 4
phases, eps = 2h, tau = eps^2, lambda = 100, 50 time steps, residual 1e-6.

The JSON line also carries
  roofline      the smoothing kernel's algorithmic bytes per launch (read u and
                rhs', write u: 12 N bytes per node) over its average launch
                time, measured with HIP events on the solve's stream;
  cpu_baseline  the FP64 oracle on one host core, timed on the first few time
                steps of the same workload and scaled to segmentations/s.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="segmentations timed")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="voronoi1024_n4")
    ap.add_argument("--schedule", choices=["fixed", "adaptive"], default="fixed",
                    help="fixed: every time step runs the cycle count found sufficient in a "
                         "calibration solve; adaptive: stop at the residual on the device")
    ap.add_argument("--cpu-sample-steps", type=int, default=6,
                    help="time steps of the oracle run for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0710_0736_amd import acseg, synth

    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    img_np, u0_np, _ = w.make(0)
    C = img_np.shape[0]
    n = w.W * w.H
    img = torch.from_numpy(img_np).to(dev)
    u0 = torch.from_numpy(u0_np).to(dev)
    u = torch.empty_like(u0)

    base = acseg.Problem.from_workload(w, C=C, levels=1, nu_pre=1, nu_post=1, max_cycles=20)

    # calibration: how many cycles does the slowest time step need?
    u.copy_(u0)
    _, _, st, _ = acseg.solve(base, img, u)
    if st["status"] != acseg.OK:
        raise RuntimeError(f"calibration solve did not converge: {st}")
    cycles = st["cycles_max"]
    if args.schedule == "fixed":
        prob = acseg.Problem(**{**base.__dict__, "max_cycles": cycles,
                                "flags": acseg.FLAG_FIXED_CYCLES})
    else:
        prob = base
    log(f"[bench] {w.name}: {w.W}x{w.H} N={w.N} C={C} steps={w.steps} tol={w.tol} "
        f"schedule={args.schedule} cycles/step<={cycles}")

    def segment():
        u.copy_(u0)
        _, c, _, _ = acseg.solve(prob, img, u, want_stats=False)
        return acseg.labels(prob, u, c)

    for _ in range(args.warmup):
        segment()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        segment()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} segmentations in {elapsed:.4f} s")

    # the timed schedule converges: check it once with statistics
    u.copy_(u0)
    _, _, st_run, _ = acseg.solve(prob, img, u)
    if st_run["status"] != acseg.OK:
        raise RuntimeError(f"benchmark schedule did not converge: {st_run}")

    roof = None
    if not args.no_roofline:
        acseg.timing_enable(True)
        acseg.timing_read()
        reps = max(2, min(args.steps, 10))
        for _ in range(reps):
            segment()
        torch.cuda.synchronize()
        t = acseg.timing_read()
        acseg.timing_enable(False)
        launches, total_ms = t["smooth"]
        avg_s = total_ms / launches / 1e3
        bytes_per_launch = 12.0 * w.N * n
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_smooth (one cycle: 2 red-black sweeps in LDS + residual)",
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
        "value": round(args.steps / elapsed, 3),
        "unit": "segmentations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "W": w.W, "H": w.H, "N": w.N, "C": C,
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
