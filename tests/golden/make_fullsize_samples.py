"""Write the full-size parity fixture (calls only the oracle and the input module).

One oracle step of the 2D Euler workload (2048 x 2048, four-quadrant data from
seed 0, transmissive, CFL 0.2, OE Type II) for k = 5 and k = 6; stores the time
step and all 12 moments of a fixed set of cells: the four corners, points along
the boundaries and the quadrant interfaces, the neighbourhood of the centre, and
300 cells drawn from numpy's PCG64 with seed 77.

Usage: python tests/golden/make_fullsize_samples.py   (about a minute per order)
"""
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fam_inputs as fi  # noqa: E402
from oracle.scheme import Config, step  # noqa: E402

N = 2048


def sample_cells(n=N):
    pts = {(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1)}
    for t in (1, 2, 3, 61, 62, 63, 64, n // 2 - 2, n // 2 - 1, n // 2, n // 2 + 1, n - 4, n - 2):
        pts |= {(t, 0), (0, t), (t, n - 1), (n - 1, t), (t, n // 2), (n // 2, t), (t, n // 2 - 1), (n // 2 - 1, t)}
    for dj in range(-3, 3):
        for di in range(-3, 3):
            pts.add((n // 2 + dj, n // 2 + di))
    rng = np.random.default_rng(77)
    for _ in range(300):
        pts.add((int(rng.integers(0, n)), int(rng.integers(0, n))))
    return np.array(sorted(pts), dtype=np.int64)   # (j, i)


def main():
    torch.set_num_threads(min(16, os.cpu_count() or 1))
    cells = sample_cells()
    out = {"cells_ji": cells}
    for k in (5, 6):
        cfg = Config(dim=2, nx=N, ny=N, k=k, system="euler", bc_x="transmissive", bc_y="transmissive",
                     oe="type2", cfl=0.2)
        U0 = torch.tensor(fi.four_quadrant(N, 0))
        U1, dt = step(U0, cfg)
        out[f"k{k}_dt"] = np.array([dt])
        out[f"k{k}_values"] = U1[:, :, cells[:, 0], cells[:, 1]].numpy()     # [4, 3, ncells]
        out[f"k{k}_avg_absmax"] = torch.abs(U1[:, 0]).amax(dim=(1, 2)).numpy()
        print(f"k={k}: dt={dt:.17g}", flush=True)
        del U1
    np.savez(os.path.join(HERE, "c3_fullsize_one_step.npz"), **out)


if __name__ == "__main__":
    main()
