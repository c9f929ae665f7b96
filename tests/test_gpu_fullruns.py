"""Full-length runs of the 1D Euler workload against a stored oracle run.

Shu-Osher-type shock / density wave, 4000 cells, k = 5, OE Type II, transmissive,
CFL 0.2, to t = 1.8 (17320 steps).  Expected values: tests/golden/shu_osher_k5_t1.8.npz,
written by tests/golden/make_shu_osher_final.py from the oracle only, together
with the oracle's own spread under 1e-16 relative input noise.  Over this many
steps the result is decided by rounding wherever the OE threshold is met by
rounding-level momentum (up to about 1e-3 relative, in most cells), so the bar
is that spread: the step count and final time must match exactly, and the
deviation from the oracle must stay within 10x the oracle's own spread, both in
the maximum and in the L1 norm of every component and moment.
"""
import os

import numpy as np
import pytest

import fam_inputs as fi
from gpu_util import both_configs, log, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "shu_osher_k5_t1.8.npz")


def test_shu_osher_run_to_final_time():
    from paper_2609_26194_amd import Fam
    gold = np.load(GOLDEN)
    _, cfg = both_configs(dim=1, nx=4000, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive",
                          oe="type2", cfl=0.2)
    fam = Fam(cfg)
    U = to_dev(fi.shu_osher(4000))
    n, t = fam.run(U, 1.8, 0)
    fam.check()
    log(f"shu-osher to t=1.8: {n} steps (oracle {int(gold['steps'])}), t = {t}")
    assert n == int(gold["steps"]) and t == float(gold["t"])
    got = U.cpu().numpy()
    ref, spread = gold["U"], gold["spread"]
    for c in range(3):
        scale = float(np.max(np.abs(ref[c, 0])))
        for m in range(2):
            dev = np.abs(got[c, m] - ref[c, m])
            log(f"  c={c} m={m}: max dev {dev.max() / scale:.2e} (oracle spread {spread[c, m].max() / scale:.2e}),"
                f" L1 dev {dev.sum() / scale:.2e} (spread {spread[c, m].sum() / scale:.2e})")
            assert dev.max() <= max(1e-12 * scale, 10 * spread[c, m].max())
            assert dev.sum() <= max(1e-12 * scale, 10 * spread[c, m].sum())
