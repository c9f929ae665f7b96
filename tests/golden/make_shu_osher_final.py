"""Write the fixture of the full 1D Euler run (calls only the oracle and the input module).

Shu-Osher-type shock / density-wave interaction on [-5, 5], 4000 cells, FAM k = 5,
OE Type II, transmissive, CFL 0.2, run to t = 1.8 with the CFL time step (last
step clipped).  Stores the final state, the step count and the oracle's own
spread: the largest change of each value over two further runs whose initial
data carry 1e-16 relative noise (the OE coefficient is scale-invariant, so
where the momentum ahead of the shock is zero up to rounding the damping is
decided by rounding; the spread measures that).

Usage: python tests/golden/make_shu_osher_final.py   (a few minutes)
"""
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fam_inputs as fi  # noqa: E402
from oracle.scheme import Config, run  # noqa: E402


def main():
    torch.set_num_threads(min(16, os.cpu_count() or 1))
    cfg = Config(dim=1, nx=4000, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive", oe="type2",
                 cfl=0.2)
    U0 = fi.shu_osher(4000)
    ref, t, n = run(torch.tensor(U0), cfg, t_final=1.8)
    ref = ref.numpy()
    env = np.zeros_like(ref)
    for seed in (0, 1):
        noise = np.random.default_rng(seed).standard_normal(U0.shape)
        pert, _, _ = run(torch.tensor(U0 * (1 + 1e-16 * noise)), cfg, t_final=1.8)
        env = np.maximum(env, np.abs(pert.numpy() - ref))
    np.savez_compressed(os.path.join(HERE, "shu_osher_k5_t1.8.npz"), U=ref, t=t, steps=n, spread=env)
    print(f"t = {t}, steps = {n}, max spread {env.max():.3e}")


if __name__ == "__main__":
    main()
