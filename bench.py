"""Benchmark of the FAM step on one MI355X.

Workload: 2D Euler (gamma = 1.4), 2048 x 2048 cells on [0,1]^2, FAM k = 5, FP64,
four-quadrant piecewise-constant data drawn from seed 0 (rho ~ U[0.1,1.5],
u, v ~ U[-1,1], p ~ U[0.02,1.5] per quadrant), transmissive boundaries, CFL 0.2,
OE Type II.  A step is the whole hot path: time step from the wave speeds,
three SSP-RK3 stages (reconstruction, Lax-Friedrichs flux, volume quadrature,
Shu-Osher update) and the OE pass.  Steps run through fam_run (replayed HIP
graphs), inputs resident in HBM before the timed region.

Prints one JSON line: the metric (cell-updates/s), a roofline object for the
dominant kernel (the RK stage kernel; its launches are timed with HIP events on
the library's own stream) and the oracle's CPU throughput on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per cell of one stage launch: stage 0 reads Us (12
# doubles) and writes Uout (12); stages 1, 2 also read U0 (12)
STAGE_BYTES = {0: 24 * 8, 1: 36 * 8, 2: 36 * 8}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--n", type=int, default=2048)
    p.add_argument("--k", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-n", type=int, default=256)
    p.add_argument("--cpu-sample-steps", type=int, default=12)
    return p.parse_args()


def stage_flops_per_cell(k):
    """Algorithmic FP64 operations of R(U) + update per cell."""
    from paper_2609_26194_amd.opcount import stage_flops
    return stage_flops(k)


def cpu_baseline(n, steps):
    """The oracle as it stands, on the same recipe at n x n for `steps` steps."""
    import torch
    import fam_inputs as fi
    from oracle.scheme import Config, step
    threads = torch.get_num_threads()
    cfg = Config(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                 oe="type2", cfl=0.2)
    U = torch.tensor(fi.four_quadrant(n, 0))
    U, _ = step(U, cfg)  # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        U, _ = step(U, cfg)
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} cells of the same workload recipe, {steps} steps ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (got --gpus {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig

    n, k = args.n, args.k
    cfg = FamConfig(dim=2, nx=n, ny=n, k=k, system="euler", bc_x="transmissive", bc_y="transmissive",
                    oe="type2", cfl=0.2)
    U0 = torch.tensor(fi.four_quadrant(n, 0), dtype=torch.float64).cuda()
    fam = Fam(cfg)
    U = U0.clone()
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup:
        fam.run(U, 0.0, args.warmup)
    U.copy_(U0)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    steps, t_sim = fam.run(U, 0.0, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cells = n * n
    value = cells * steps / elapsed

    # dominant kernel: the RK stage kernel, timed per launch with HIP events on
    # the library's stream, same launch configuration as inside the steps
    dtd = fam.dt(U)
    W1, W2 = torch.empty_like(U), torch.empty_like(U)
    reps = 10
    durs = {0: [], 1: [], 2: []}
    ins = {0: (U, U, W1), 1: (U, W1, W2), 2: (U, W2, W1)}
    for rep in range(reps + 1):
        fam.dt(U)
        for s in range(3):
            U0_, Us_, Uo_ = ins[s]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fam.stream.wait_stream(torch.cuda.current_stream())
            e0.record(fam.stream)
            from paper_2609_26194_amd.fam import fam_stage
            fam_stage(fam.h, s, U0_, Us_, Uo_, dtd)
            e1.record(fam.stream)
            torch.cuda.current_stream().wait_stream(fam.stream)
            e1.synchronize()
            if rep > 0:
                durs[s].append(e0.elapsed_time(e1) * 1e-3)
    avg = {s: sum(v) / len(v) for s, v in durs.items()}
    # stage 1 (the middle stage) is the representative launch: reads Us and U0, writes Uout
    dur = avg[1]
    flops = stage_flops_per_cell(k) * cells
    achieved_tflops = flops / dur / 1e12
    bytes_alg = STAGE_BYTES[1] * cells
    achieved_gbs = bytes_alg / dur / 1e9
    roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / FP64_PEAK_TFLOPS, "traffic": None,
                "kernel": "stage2d_kernel<5, Euler<2>> (RK stage 2 of 3)",
                "launch_ms": dur * 1e3, "hbm_algorithmic_GBs": achieved_gbs,
                "hbm_algorithmic_frac": achieved_gbs / HBM_PEAK_GBS,
                "stage_launch_ms": [avg[0] * 1e3, avg[1] * 1e3, avg[2] * 1e3]}
    step_bytes = 928 * cells
    out = {
        "metric": "2D Euler FAM cell-updates/s (FP64, k=5)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Euler four-quadrant (seed 0) {n}x{n}, FAM k={k}, OE Type II, "
                               f"transmissive, CFL 0.2", "cells": cells, "k": k,
                   "step_algorithmic_GBs": step_bytes * steps / elapsed / 1e9},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_sample_steps)
    fam.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
