"""Benchmark of the FAM step on one MI355X.

Main workload: 2D Euler (gamma = 1.4), 2048 x 2048 cells on [0,1]^2, FAM k = 5,
FP64, four-quadrant piecewise-constant data drawn from seed 0 (rho ~ U[0.1,1.5],
u, v ~ U[-1,1], p ~ U[0.02,1.5] per quadrant), transmissive boundaries, CFL 0.2,
OE Type II, positivity limiter on (without it this data leaves the admissible
set within 60-70 steps at k = 5; the limiter is the identity in every cell whose
flux points are all admissible).  A step is the whole hot path: time step from the wave speeds, three
SSP-RK3 stages (reconstruction, Lax-Friedrichs flux, volume quadrature,
Shu-Osher update) and the OE pass.  Steps run through fam_run (replayed HIP
graphs), inputs resident in HBM before the timed region.

Prints one JSON line with the metric (cell-updates/s), a roofline object for the
dominant kernel (the RK stage kernel, its launches timed with HIP events on the
library's own stream), the oracle's CPU throughput on a bounded sample, and two
sub-measurements: the same workload at k = 6, the batched workload (256 uneven
instances in one persistent launch per stage against one context per instance)
and the adjoint workload (gradient cost over forward cost at 1024^2, 400 steps,
checkpoint every 20).

``python bench.py --ingest-counters FETCH.csv WRITE.csv`` turns the per-dispatch
CSVs of two ``rocprofv3 --pmc`` runs of this script (FETCH_SIZE, then
WRITE_SIZE) into profiles/stage2d_k5_2048_counters.json: HBM bytes per stage
launch, scaled by what the same counters read for the 1 GiB streaming copy this
script performs, with a hash of the stage kernel's sources so that the figure is
dropped (traffic null) once the kernel changes.
"""
import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per cell of one stage launch: stage 0 reads Us (12
# doubles) and writes Uout (12); stages 1, 2 also read U0 (12)
STAGE_BYTES = {0: 24 * 8, 1: 36 * 8, 2: 36 * 8}
OE_BYTES = 20 * 8                 # OE reads the 12 moments, writes the 8 first moments
STEP_BYTES = sum(STAGE_BYTES.values()) + OE_BYTES   # 928 B per cell-update
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # 256 CUs x 2.4 GHz x 128 FP64 flops / clock
COPY_BYTES = 1 << 30             # calibration copy for the HBM counters
COUNTERS_JSON = os.path.join(ROOT, "profiles", "stage2d_k5_2048_counters.json")
STAGE_SOURCES = ["fam_kernels2d.hip", "fam_device.h", "fam_eval.h", "fam_kernels.h", "fam_strip.h"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1, help="number of GPUs (only 1: the library runs a mesh or a batch on one GPU)")
    p.add_argument("--steps", type=int, default=200, help="timed steps of the main workload")
    p.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed region")
    p.add_argument("--n", type=int, default=2048, help="mesh size n x n of the main workload")
    p.add_argument("--k", type=int, default=5, help="order of the main workload")
    p.add_argument("--no-main", action="store_true", help="skip the main workload (profiling of the other legs)")
    p.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle baseline on the host")
    p.add_argument("--cpu-sample-n", type=int, default=512, help="mesh size of the oracle baseline sample")
    p.add_argument("--cpu-sample-steps", type=int, default=24, help="steps of the oracle baseline sample")
    p.add_argument("--no-k6", action="store_true", help="skip the k = 6 run of the main workload")
    p.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    p.add_argument("--batched-steps", type=int, default=100, help="steps of the batched workload")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    p.add_argument("--adjoint-n", type=int, default=1024, help="mesh size of the adjoint workload")
    p.add_argument("--adjoint-steps", type=int, default=400, help="steps of the adjoint workload")
    p.add_argument("--adjoint-checkpoint", type=int, default=20, help="checkpoint spacing of the adjoint workload")
    p.add_argument("--no-dmr", action="store_true", help="skip the double Mach reflection run")
    p.add_argument("--dmr-t", type=float, default=0.2, help="final time of the double Mach reflection run")
    p.add_argument("--dmr-cfl", type=float, default=0.55, help="CFL number of the double Mach reflection run "
                   "(the paper's FAM5 discontinuous tests: 0.55)")
    p.add_argument("--no-char", action="store_true", help="skip the characteristic-variable comparison")
    p.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), help="record the HBM traffic of the stage kernel from two rocprofv3 counter CSVs")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_sources_hash():
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_26194_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# HBM counters
# ---------------------------------------------------------------------------
def _per_dispatch(path, counter):
    """{kernel name: [value per dispatch]} from a rocprofv3 counter_collection CSV."""
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def ingest_counters(fetch_csv, write_csv):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, key):
        names = [n for n in d if key in n]
        if not names:
            raise SystemExit(f"no dispatch of a kernel matching {key!r}")
        return [v for n in names for v in d[n]]

    # the stage kernel that the timed launches use: the segment-list kernel when
    # the autotuner chose it, else the fixed-height one
    key = "stage2d_list_kernel<5" if any("stage2d_list_kernel<5" in n for n in fetch) else "stage2d_kernel<5"
    stage_f = pick(fetch, key)
    stage_w = pick(write, key)
    copy_f = max(pick(fetch, "Mul"))
    copy_w = max(pick(write, "Mul"))
    kib = COPY_BYTES / 1024.0
    f_scale, w_scale = kib / copy_f, kib / copy_w
    fetch_b = sum(stage_f) / len(stage_f) * 1024.0 * f_scale
    write_b = sum(stage_w) / len(stage_w) * 1024.0 * w_scale
    rec = {"kernel": f"{key}, Euler<2>...> (all three RK stages)", "kernel_key": key,
           "workload": "2D Euler four-quadrant 2048x2048, k=5, positivity limiter",
           "dispatches": len(stage_f),
           "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
           "traffic_bytes_per_launch": fetch_b + write_b,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": copy_f, "write_kib": copy_w,
                                "fetch_scale": f_scale, "write_scale": w_scale},
           "kernel_sources_sha256": stage_sources_hash()}
    os.makedirs(os.path.dirname(COUNTERS_JSON), exist_ok=True)
    with open(COUNTERS_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def stored_traffic(key):
    """HBM bytes per stage launch of kernel `key` from the committed counters, or None if
    they are stale or were taken on the other stage kernel."""
    try:
        with open(COUNTERS_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != stage_sources_hash() or rec.get("kernel_key") != key:
        return None
    return rec.get("traffic_bytes_per_launch")


# ---------------------------------------------------------------------------
# measurements
# ---------------------------------------------------------------------------
def host_cpus():
    """(threads to use, visible CPUs, CPU model): all CPUs this process may run on, capped by
    OMP_NUM_THREADS when it is set (a host's share for one job)."""
    visible = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = visible
    cap = os.environ.get("OMP_NUM_THREADS")
    threads = min(usable, int(cap)) if cap and cap.isdigit() and int(cap) > 0 else usable
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, visible, usable, model


def cpu_baseline(n, steps):
    """The oracle as it stands, on the same recipe at n x n for `steps` steps, with every host
    thread this job may use, and on one thread for a smaller sample."""
    import torch
    import fam_inputs as fi
    from oracle.scheme import Config, step
    threads, visible, usable, model = host_cpus()
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    cfg = Config(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                 oe="type2", cfl=0.2, pp=True)
    try:
        U = torch.tensor(fi.four_quadrant(n, 0))
        U, _ = step(U, cfg)  # warm-up
        t0 = time.perf_counter()
        for _ in range(steps):
            U, _ = step(U, cfg)
        dt = time.perf_counter() - t0
        # the same oracle on one thread (a smaller sample of the same recipe)
        n1, steps1 = 256, 2
        cfg1 = Config(dim=2, nx=n1, ny=n1, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                      oe="type2", cfl=0.2, pp=True)
        torch.set_num_threads(1)
        V, _ = step(torch.tensor(fi.four_quadrant(n1, 0)), cfg1)  # warm-up
        t1 = time.perf_counter()
        for _ in range(steps1):
            V, _ = step(V, cfg1)
        dt1 = time.perf_counter() - t1
    finally:
        torch.set_num_threads(prev)
    return {"value": n * n * steps / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} cells of the same workload recipe, {steps} steps after one warm-up step "
                      f"({dt:.1f} s)",
            "host": {"cpu_model": model, "nproc": visible, "usable_cpus": usable,
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")},
            "single_thread": {"value": n1 * n1 * steps1 / dt1, "cores": 1,
                              "sample": f"{n1}x{n1} cells, {steps1} steps after one warm-up step ({dt1:.1f} s)"}}


def timed_launches(fam, calls, reps):
    """Back-to-back launches of calls (a list of (key, fn)) on the library stream, reps + 1
    times, each bracketed by a HIP event pair on that stream; one host synchronisation at the
    end, so the device stays busy as in a run.  Returns {key: [seconds per launch]} without
    the first repetition."""
    import torch
    ev = []
    fam.stream.wait_stream(torch.cuda.current_stream())
    for rep in range(reps + 1):
        for key, fn in calls:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(fam.stream)
            fn()
            e1.record(fam.stream)
            ev.append((rep, key, e0, e1))
    torch.cuda.current_stream().wait_stream(fam.stream)
    ev[-1][3].synchronize()
    out = {}
    for rep, key, e0, e1 in ev:
        if rep > 0:
            out.setdefault(key, []).append(e0.elapsed_time(e1) * 1e-3)
    return out


def stage_roofline(fam, U, k, cells, seg_list, reps=10):
    """Per-launch duration of the three RK stage launches, HIP events on the library stream."""
    import torch
    from paper_2609_26194_amd.fam import fam_stage
    dtd = fam.dt(U)
    W1, W2 = torch.empty_like(U), torch.empty_like(U)
    calls = [(0, lambda: fam_stage(fam.h, 0, U, U, W1, dtd)), (1, lambda: fam_stage(fam.h, 1, U, W1, W2, dtd)),
             (2, lambda: fam_stage(fam.h, 2, U, W2, W1, dtd))]
    durs = timed_launches(fam, calls, reps)
    avg = {s: sum(v) / len(v) for s, v in durs.items()}
    dur = sum(avg.values()) / 3.0
    from paper_2609_26194_amd.opcount import stage_flops
    achieved = stage_flops(k) * cells / dur / 1e12
    bytes_alg = sum(STAGE_BYTES.values()) / 3.0 * cells
    gbs = bytes_alg / dur / 1e9
    key = f"stage2d_list_kernel<{k}" if seg_list else f"stage2d_kernel<{k}"
    traffic = stored_traffic(key)
    if seg_list:
        kernel = (f"stage2d_list_kernel<{k}, Euler<2>> (mean of the three RK stage launches; as in a step, "
                  f"the stage-0 launch also re-cuts the segment list: part_scan_kernel, part_cut_kernel)")
    else:
        kernel = (f"stage2d_kernel<{k}, Euler<2>, true> and its tile_order_kernel (mean of the three RK "
                  f"stage launches)")
    return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
            "kernel": kernel,
            "launch_ms": dur * 1e3, "stage_launch_ms": [avg[s] * 1e3 for s in range(3)],
            "flops_per_cell": stage_flops(k), "algorithmic_bytes_per_launch": bytes_alg,
            "hbm_algorithmic_GBs": gbs, "hbm_algorithmic_frac": gbs / HBM_PEAK_GBS}


def oe_roofline(fam, U, k, cells, reps=10):
    """The OE kernel's launch through fam_oe (which writes all 12 planes: 192 B per cell; the
    step's own OE writes the 8 moment planes, 160 B), on the pre-OE state of one step from U,
    HIP events on the library stream."""
    import torch
    from paper_2609_26194_amd.fam import fam_oe, fam_stage
    from paper_2609_26194_amd.opcount import oe_flops
    dtd = fam.dt(U)
    W1, W2, W3 = torch.empty_like(U), torch.empty_like(U), torch.empty_like(U)
    fam_stage(fam.h, 0, U, U, W1, dtd)
    fam_stage(fam.h, 1, U, W1, W2, dtd)
    fam_stage(fam.h, 2, U, W2, W3, dtd)
    durs = timed_launches(fam, [("oe", lambda: fam_oe(fam.h, W3, W1, dtd))], reps)["oe"]
    dur = sum(durs) / len(durs)
    bytes_alg = 24 * 8 * cells
    gbs = bytes_alg / dur / 1e9
    return {"kernel": f"oe2d_kernel<{k}, Euler<2>> through fam_oe (12 planes written)", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "launch_ms": dur * 1e3, "algorithmic_bytes_per_launch": bytes_alg,
            "flops_per_cell": oe_flops(k)}


def copy_calibration():
    """One plain streaming kernel that reads COPY_BYTES and writes COPY_BYTES (y = 1.0 * x),
    the HBM-counter calibration.  The buffers exceed the 256 MB last-level cache and a
    512 MiB fill runs in between, so the read comes from HBM."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    flush = torch.empty(512 << 17, dtype=torch.float64, device="cuda")
    flush.fill_(0.0)
    torch.cuda.synchronize()
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del flush


def batched(steps):
    """Batched workload: 256 square instances (sizes from seed 1, data seeds 1000 + i), k = 5,
    OE Type II, positivity limiter on, transmissive; one persistent launch per stage against
    one context per instance."""
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    sizes = fi.batch_sizes(256, 1)
    cfgs = [FamConfig(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                      oe="type2", cfl=0.2, pp=True) for n in sizes]
    cells = sum(n * n for n in sizes)
    states = [torch.tensor(fi.batch_instance(i, n), dtype=torch.float64).cuda() for i, n in enumerate(sizes)]
    bat = Fam(cfgs[0], batch=cfgs)
    offs = bat.offsets()
    U0 = torch.zeros(bat.len, dtype=torch.float64, device="cuda")
    for o, s in zip(offs, states):
        U0[o:o + s.numel()] = s.reshape(-1)
    tuned = bat.autotune(U0)
    U = U0.clone()
    bat.run(U, 0.0, 4)
    U.copy_(U0)
    bat.set_time(0.0)   # the clock back to the initial state's time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bat.run(U, 0.0, steps)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    bat.close()
    # one context per instance, each advanced with its own graph-replayed fam_run
    singles = [Fam(c) for c in cfgs]
    work = [s.clone() for s in states]
    for f, w in zip(singles, work):
        f.autotune(w, reps=2)
        f.run(w, 0.0, 4)
    for w, s in zip(work, states):
        w.copy_(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f, w in zip(singles, work):
        f.run(w, 0.0, steps)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    same = all(torch.equal(U[o:o + w.numel()], w.reshape(-1)) for o, w in zip(offs, work))
    for f in singles:
        f.close()
    return {"workload": "256 instances, sizes U{64..512} (seed 1), four-quadrant data (seeds 1000+i), "
                        f"k=5, OE Type II, positivity limiter, {steps} steps",
            "cells": cells, "batched_cell_updates_per_s": cells * steps / t_b,
            "per_instance_cell_updates_per_s": cells * steps / t_s,
            "speedup": t_s / t_b, "batched_ms_per_step": t_b / steps * 1e3,
            "per_instance_ms_per_step": t_s / steps * 1e3, "bitwise_equal": bool(same),
            "autotuned": {"tile_height": tuned[0], "persistent_blocks": tuned[1]}}


def adjoint(n, steps, every):
    """Adjoint workload: periodic density waves (seed 2) on n x n, k = 5, OE Type II,
    fixed dt = half the CFL step of the initial state; gradient of the window functional."""
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    cfg = FamConfig(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="periodic", bc_y="periodic",
                    oe="type2", cfl=0.2)
    fam = Fam(cfg)
    U0 = torch.tensor(fi.density_waves(n), dtype=torch.float64).cuda()
    fam.autotune(U0)
    dt = 0.5 * float(fam.dt(U0)[0])
    U = U0.clone()
    fam.run(U, 0.0, 10, dt)
    fam.adjoint(U0, every, dt, every)
    U.copy_(U0)
    fam.set_time(0.0)   # the clock back to the initial state's time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fam.run(U, 0.0, steps, dt)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    J, g = fam.adjoint(U0, steps, dt, every)
    torch.cuda.synchronize()
    t_a = time.perf_counter() - t0
    out = {"workload": f"2D Euler periodic density waves (seed 2) {n}x{n}, k=5, OE Type II, {steps} steps, "
                       f"checkpoint every {every}", "J": J,
           "forward_ms": t_f * 1e3, "gradient_ms": t_a * 1e3, "gradient_over_forward": t_a / t_f}
    # the whole run's tape resident in HBM (4 states per step: 161 GB at 1024^2 x 400 steps):
    # one segment, no recomputation; the same gradient bit for bit
    from paper_2609_26194_amd.fam import FamError
    tape_gb = 4 * steps * U0.numel() * 8 / 1e9
    try:
        fam.adjoint(U0, steps, dt, steps)   # allocates the tape, warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J2, g2 = fam.adjoint(U0, steps, dt, steps)
        torch.cuda.synchronize()
        t_r = time.perf_counter() - t0
        out["tape_resident"] = {"tape_GB": tape_gb, "gradient_ms": t_r * 1e3, "gradient_over_forward": t_r / t_f,
                                "same_gradient_bitwise": bool(torch.equal(g, g2)) and J == J2}
    except FamError as e:
        out["tape_resident"] = {"tape_GB": tape_gb, "skipped": str(e)}
    fam.close()
    return out


def k6_leg(n, steps, warmup):
    """The main workload at k = 6 (same data, limiter, boundaries): cell-updates/s only."""
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    cfg = FamConfig(dim=2, nx=n, ny=n, k=6, system="euler", bc_x="transmissive", bc_y="transmissive",
                    oe="type2", cfl=0.2, pp=True)
    U0 = torch.tensor(fi.four_quadrant(n, 0), dtype=torch.float64).cuda()
    fam = Fam(cfg)
    tuned = fam.autotune(U0)
    U = U0.clone()
    if warmup:
        fam.run(U, 0.0, warmup)
    U.copy_(U0)
    fam.set_time(0.0)   # the clock back to the initial state's time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, _ = fam.run(U, 0.0, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fam.close()
    return {"workload": f"2D Euler four-quadrant (seed 0) {n}x{n}, FAM k=6, OE Type II (jumps of p6), "
                        f"transmissive, CFL 0.2, positivity limiter, {done} steps",
            "cell_updates_per_s": n * n * done / elapsed, "ms_per_step": elapsed / done * 1e3,
            "autotuned_tile_heights": {"stage": tuned[0], "oe": tuned[1]}}


def launch_split(fam, U, reps=10):
    """Standalone launches of one step at the state U: the three RK stage launches and
    the OE launch, each bracketed by HIP events on the library stream (ms, averaged)."""
    import torch
    from paper_2609_26194_amd.fam import fam_oe, fam_stage
    dtd = fam.dt(U)
    W1, W2, W3 = torch.empty_like(U), torch.empty_like(U), torch.empty_like(U)
    calls = [("stage", lambda: fam_stage(fam.h, 0, U, U, W1, dtd)), ("stage", lambda: fam_stage(fam.h, 1, U, W1, W2, dtd)),
             ("stage", lambda: fam_stage(fam.h, 2, U, W2, W3, dtd)), ("oe", lambda: fam_oe(fam.h, W3, W1, dtd))]
    durs = timed_launches(fam, calls, reps)
    # per step: the three stage launches summed, the OE launch (ms)
    return {"stage": sum(durs["stage"]) / reps * 1e3, "oe": sum(durs["oe"]) / reps * 1e3}


def char_leg(so_n=4000, so_steps=2000, dmr_steps=1000):
    """Conservative against local characteristic variables for FAM5, the comparison of Table
    runtime-main Panel B: a Shu-Osher-type 1D run ([-5, 5], OE Type II, CFL 0.2) and the double
    Mach reflection (1440 x 480, limiter).  Each variant runs the same number of steps from the
    same data (both tile heights autotuned in 2D); reported: ms per step (graph-replayed steps),
    the RK stage launches (reconstruction, fluxes, quadrature: where the transform sits) and the
    OE launch of one step at the final state, and the ratios characteristic / conservative."""
    import dataclasses
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    cases = [
        ("shu_osher", FamConfig(dim=1, nx=so_n, x0=-5.0, x1=5.0, k=5, system="euler", oe="type2", cfl=0.2,
                                bc_x="transmissive"), fi.shu_osher(so_n), so_steps, so_n),
        ("double_mach", FamConfig(dim=2, nx=1440, ny=480, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler",
                                  oe="type2", cfl=0.2, pp=True, dmr=True), fi.double_mach(1440, 480), dmr_steps,
         1440 * 480),
    ]
    res = {}
    for name, cfg, U0h, nsteps, cells in cases:
        U0 = torch.tensor(U0h, dtype=torch.float64).cuda()
        row = {"cells": cells, "steps": nsteps}
        for cv in (False, True):
            fam = Fam(dataclasses.replace(cfg, char_vars=cv))
            if cfg.dim == 2:
                fam.autotune(U0)
            U = U0.clone()
            fam.run(U, 0.0, 5)   # warm-up
            U.copy_(U0)
            fam.set_time(0.0)   # the clock back to the initial state's time
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            steps, _ = fam.run(U, 0.0, nsteps)
            torch.cuda.synchronize()
            elapsed = time.perf_counter() - t0
            fam.check()
            split = launch_split(fam, U)
            fam.close()
            row["characteristic" if cv else "conservative"] = {
                "ms_per_step": elapsed / steps * 1e3, "cell_updates_per_s": cells * steps / elapsed,
                "stage_launch_ms": split["stage"], "oe_launch_ms": split["oe"]}
        c, w = row["conservative"], row["characteristic"]
        row["ratio"] = {"total": w["ms_per_step"] / c["ms_per_step"],
                        "stages": w["stage_launch_ms"] / c["stage_launch_ms"],
                        "oe": w["oe_launch_ms"] / c["oe_launch_ms"]}
        res[name] = row
    return res


def dmr_leg(t_final, cfl, nx=1440, ny=480):
    """The paper's double Mach reflection run: [0, 3] x [0, 1], 1440 x 480, FAM5, OE Type II,
    positivity limiter, to t_final at C = cfl (the paper's FAM5 discontinuous tests use 0.55,
    Sec. 4, time stepping); cell-updates/s, the step count, and the split of one step's time
    between the three RK stage launches and the OE launch (HIP events on the library stream,
    at the final state)."""
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    cfg = FamConfig(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2",
                    cfl=cfl, pp=True, dmr=True)
    U0 = torch.tensor(fi.double_mach(nx, ny), dtype=torch.float64).cuda()
    fam = Fam(cfg)
    tuned = fam.autotune(U0)
    U = U0.clone()
    fam.run(U, 0.0, 5)   # warm-up
    U.copy_(U0)
    fam.set_time(0.0)   # the clock back to the initial state's time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, t = fam.run(U, t_final, 10 ** 7)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fam.check()
    tot = launch_split(fam, U)
    fam.close()
    return {"workload": f"double Mach reflection {nx}x{ny} on [0,3]x[0,1], FAM5, OE Type II, positivity limiter, "
                        f"CFL {cfl}, to t = {t:.4f}", "cfl": cfl, "steps": steps,
            "cell_updates_per_s": nx * ny * steps / elapsed,
            "ms_per_step": elapsed / steps * 1e3, "seconds": elapsed,
            # standalone launches of one step (each stage launch re-cuts its segment list; inside the
            # graph-replayed step that happens once), and the OE's share of them
            "launch_ms": {"rk_stages": tot["stage"], "oe": tot["oe"]},
            "oe_fraction": tot["oe"] / (tot["stage"] + tot["oe"]),
            "autotuned_tile_heights": {"stage": tuned[0], "oe": tuned[1]}}


def main_workload(args, n, k):
    """The headline measurement: cell-updates/s of the full step and the stage-kernel roofline."""
    import torch
    import fam_inputs as fi
    from paper_2609_26194_amd import Fam, FamConfig
    cfg = FamConfig(dim=2, nx=n, ny=n, k=k, system="euler", bc_x="transmissive", bc_y="transmissive",
                    oe="type2", cfl=0.2, pp=True)
    U0 = torch.tensor(fi.four_quadrant(n, 0), dtype=torch.float64).cuda()
    fam = Fam(cfg)
    tuned = fam.autotune(U0)
    log(f"autotuned strip-tile heights: stage {tuned[0]}, OE {tuned[1]}")
    U = U0.clone()
    log(f"warmup {args.warmup} steps")
    if args.warmup:
        fam.run(U, 0.0, args.warmup)
    U.copy_(U0)
    fam.set_time(0.0)   # the clock back to the initial state's time
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    steps, t_sim = fam.run(U, 0.0, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cells = n * n
    value = cells * steps / elapsed
    log("stage launches")
    roofline = stage_roofline(fam, U, k, cells, seg_list=tuned[0] == 0)
    log("OE launches")
    oe_roof = oe_roofline(fam, U, k, cells)
    fam.close()
    copy_calibration()
    # the whole step's algorithmic HBM rate: cell-updates/s x 928 B (three stages and the OE)
    roofline["step_algorithmic_GBs"] = value * STEP_BYTES / 1e9
    roofline["step_algorithmic_frac"] = value * STEP_BYTES / 1e9 / HBM_PEAK_GBS
    return {
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
                               f"transmissive, CFL 0.2, positivity limiter", "cells": cells, "k": k, "t_simulated": t_sim,
                   "autotuned_tile_heights": {"stage": tuned[0], "oe": tuned[1]}},
        "roofline": roofline,
        "oe_roofline": oe_roof,
    }


def main():
    args = parse()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the library runs a mesh or a batch on a "
              f"single GPU", file=sys.stderr)
        sys.exit(2)
    n, k = args.n, args.k
    out = {}
    if not args.no_main:
        out = main_workload(args, n, k)
    if not args.no_main and not args.no_k6:
        log("k = 6 workload")
        out["k6"] = k6_leg(n, args.steps, args.warmup)
    if not args.no_batched:
        log("batched workload")
        out["batched"] = batched(args.batched_steps)
    if not args.no_dmr:
        log("double Mach reflection")
        out["dmr"] = dmr_leg(args.dmr_t, args.dmr_cfl)
    if not args.no_char:
        log("characteristic variables")
        out["characteristic_variables"] = char_leg()
    if not args.no_adjoint:
        log("adjoint workload")
        out["adjoint"] = adjoint(args.adjoint_n, args.adjoint_steps, args.adjoint_checkpoint)
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_sample_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
