"""Parity on seeded random configurations: mesh sizes ragged against the strips and row tiles
(3..190 cells per direction), every order k = 3..6, the three systems, periodic and transmissive
boundaries in each direction, OE off / Type I / Type II, the positivity limiter on some Euler
cases, 1D and 2D.  Each case runs two steps of fam_run (CFL time step) on the GPU and of the
oracle from the same seeded state; the bar is the parity bar, relative L-infinity 1e-12.
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
TOL = 1e-12
NCASES = 36


def _case(i):
    rng = np.random.default_rng(5000 + i)
    dim = 1 if i % 6 == 5 else 2
    system = ("advection", "burgers", "euler", "euler")[i % 4]
    k = int(rng.integers(3, 7))
    nx = int(rng.integers(3, 191))
    ny = int(rng.integers(3, 151)) if dim == 2 else 1
    bcs = ("periodic", "transmissive")
    bc_x, bc_y = bcs[int(rng.integers(2))], bcs[int(rng.integers(2))]
    oe = ("off", "type1", "type2")[int(rng.integers(3))]
    pp = system == "euler" and dim == 2 and bool(rng.integers(2))
    kw = dict(dim=dim, nx=nx, k=k, system=system, bc_x=bc_x, oe=oe, cfl=0.2)
    if dim == 2:
        kw.update(ny=ny, bc_y=bc_y, pp=pp)
    if system == "advection":
        kw.update(a=(0.8, -0.5) if dim == 2 else (1.0, 0.0))
    seed = 6000 + i
    if system == "euler" and dim == 2:
        U0 = fi.four_quadrant(nx, seed, ny=ny) if pp else fi.random_euler_state_2d(nx, ny, seed, amp=0.2)
    elif system == "euler":
        U0 = fi.smooth_euler_1d(nx)
    else:
        shape = (1, 3, ny, nx) if dim == 2 else (1, 2, nx)
        U0 = fi.random_state(shape, seed, 0.2, 1.2)
    return kw, U0


@pytest.mark.parametrize("i", range(NCASES))
def test_random_configuration_two_steps(i):
    kw, U0 = _case(i)
    log(f"  case {i}: {kw}")
    ora, cfg = both_configs(**kw)
    ref, _, steps = S.run(torch.tensor(U0), ora, nsteps=2)
    assert steps == 2
    from paper_2609_26194_amd import Fam
    fam = Fam(cfg)
    U = to_dev(U0)
    done, _ = fam.run(U, 0.0, 2)
    fam.check()
    fam.close()
    assert done == 2
    err = rel_linf(U, ref)
    log(f"    rel Linf {err:.2e}")
    assert err <= TOL
