"""Write the full-size fixture of the limiter runs (calls only the oracle and the input module).

One oracle step of each of:

* the 2D Euler four-quadrant workload (2048 x 2048, seed 0, transmissive, CFL 0.2, OE
  Type II, k = 5 and k = 6) with the positivity limiter on, as the benchmark runs it;
* the double Mach reflection at the paper's size (1440 x 480 on [0, 3] x [0, 1], k = 5,
  OE Type II, limiter, CFL 0.2) from t = 0.

Stored per case: the time step and all 12 moments of a fixed set of cells (corners,
boundary rows and columns, the discontinuities of the initial data, 300 cells from
numpy's PCG64 with seed 78) plus up to 256 cells, in the order of their linear
index, whose stage-0 reconstruction the oracle's limiter scales (theta < 1).

Usage: python tests/golden/make_fullsize_limiter_samples.py   (about five minutes)
"""
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fam_inputs as fi  # noqa: E402
import oracle.scheme as S  # noqa: E402


def base_cells(nx, ny, lines_x, lines_y, seed):
    pts = {(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)}
    for t in (1, 2, 3, 61, 62, 63, 64, nx // 2, nx - 4, nx - 2):
        if t < nx:
            pts |= {(0, t), (1, t), (ny - 1, t), (ny - 2, t)}
    for t in (1, 2, 3, ny // 2, ny - 4, ny - 2):
        pts |= {(t, 0), (t, 1), (t, nx - 1), (t, nx - 2)}
    for x in lines_x:
        for j in (0, 1, ny // 3, ny // 2, ny - 1):
            for di in (-2, -1, 0, 1):
                if 0 <= x + di < nx:
                    pts.add((j, x + di))
    for y in lines_y:
        for i in (0, 1, nx // 3, nx // 2, nx - 1):
            for dj in (-2, -1, 0, 1):
                if 0 <= y + dj < ny:
                    pts.add((y + dj, i))
    rng = np.random.default_rng(seed)
    for _ in range(300):
        pts.add((int(rng.integers(0, ny)), int(rng.integers(0, nx))))
    return pts


def limited_cells(U, cfg, t=0.0, cap=256):
    Upad = S.pad(U, cfg, t=t)
    monos, coef = S.reconstruct_stage(Upad, cfg)
    vals = S.point_values(monos, coef, S.points_2d())
    avg = Upad[:, 0, 1:-1, 1:-1]
    th1, th2 = S.pp_theta(vals, avg, cfg.phys)
    lim = ((th1 < 1) | (th2 < 1))[1:-1, 1:-1]          # interior cells
    js, is_ = torch.nonzero(lim, as_tuple=True)
    return {(int(j), int(i)) for j, i in zip(js[:cap].tolist(), is_[:cap].tolist())}, int(lim.sum())


def run_case(cfg, U0, lines_x, lines_y, seed):
    lim, nlim = limited_cells(U0, cfg)
    cells = np.array(sorted(base_cells(cfg.nx, cfg.ny, lines_x, lines_y, seed) | lim), dtype=np.int64)
    U1, dt = S.step(U0, cfg, t=0.0)
    print(f"  dt = {dt:.17g}, {nlim} limited cells at stage 0, {len(cells)} sampled", flush=True)
    return {"cells_ji": cells, "dt": np.array([dt]), "values": U1[:, :, cells[:, 0], cells[:, 1]].numpy(),
            "avg_absmax": torch.abs(U1[:, 0]).amax(dim=(1, 2)).numpy(), "n_limited_stage0": np.array([nlim])}


def main():
    torch.set_num_threads(min(16, os.cpu_count() or 1))
    out = {}
    print("four-quadrant 2048^2, k = 5, limiter", flush=True)
    cfg = S.Config(dim=2, nx=2048, ny=2048, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                   oe="type2", cfl=0.2, pp=True)
    for key, v in run_case(cfg, torch.tensor(fi.four_quadrant(2048, 0)), (1024,), (1024,), 78).items():
        out["c3pp_" + key] = v
    print("four-quadrant 2048^2, k = 6, limiter", flush=True)
    cfg = S.Config(dim=2, nx=2048, ny=2048, k=6, system="euler", bc_x="transmissive", bc_y="transmissive",
                   oe="type2", cfl=0.2, pp=True)
    for key, v in run_case(cfg, torch.tensor(fi.four_quadrant(2048, 0)), (1024,), (1024,), 78).items():
        out["c3pp6_" + key] = v
    print("double Mach reflection 1440 x 480, k = 5, limiter", flush=True)
    cfg = S.Config(dim=2, nx=1440, ny=480, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2",
                   cfl=0.2, pp=True, dmr=True)
    # the initial shock meets the bottom at x = 1/6 (cell 80) and leans right with height
    for key, v in run_case(cfg, torch.tensor(fi.double_mach(1440, 480)), (80, 240, 400), (), 79).items():
        out["dmr_" + key] = v
    np.savez(os.path.join(HERE, "fullsize_limiter_one_step.npz"), **out)


if __name__ == "__main__":
    main()
