"""The adjoint (fam_adjoint) on seeded random configurations: ragged periodic meshes of 9..100 x
9..80 cells (against the 16 x 16 tiles of the reverse kernels), orders k = 3..6, OE Type II or off,
2..4 fixed-dt steps and a checkpoint spacing of 1..nsteps, on tie-free random states.  The
functional and its gradient against the oracle's reverse-mode gradient of the same steps, at the
bars of the adjoint tests: J to 1e-12 relative, dJ/dU0 to 1e-10 of its largest entry.
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.functional as OF
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
NCASES = 8


def _case(i):
    rng = np.random.default_rng(9900 + i)
    k = int(rng.integers(3, 7))
    oe = ("type2", "off")[int(rng.integers(2))]
    nx, ny = int(rng.integers(9, 101)), int(rng.integers(9, 81))
    nsteps = int(rng.integers(2, 5))
    every = int(rng.integers(1, nsteps + 1))
    return dict(k=k, oe=oe, nx=nx, ny=ny, nsteps=nsteps, every=every, seed=9950 + i)


@pytest.mark.parametrize("i", range(NCASES))
def test_random_adjoint_matches_oracle_gradient(i):
    from paper_2609_26194_amd import Fam
    c = _case(i)
    log(f"  adjoint case {i}: {c}")
    ora, cfg = both_configs(dim=2, nx=c["nx"], ny=c["ny"], k=c["k"], system="euler", bc_x="periodic",
                            bc_y="periodic", oe=c["oe"], cfl=0.2)
    U0 = fi.random_euler_state_2d(c["nx"], c["ny"], c["seed"], amp=0.1)
    dt = 0.5 * S.cfl_dt(torch.tensor(U0), ora)
    J_ref, g_ref = OF.reference_gradient(U0, ora, c["nsteps"], dt)
    fam = Fam(cfg)
    J, g = fam.adjoint(to_dev(U0), c["nsteps"], dt, c["every"])
    fam.close()
    g = g.cpu()
    err = float((g - g_ref).abs().max()) / float(g_ref.abs().max())
    log(f"    J rel {abs(J - J_ref) / abs(J_ref):.2e}, grad rel Linf {err:.2e}")
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
    assert err <= 1e-10
