"""Parity of batched contexts on seeded random batches: 3 to 6 2D instances per batch with ragged
rectangular meshes (3..120 cells per direction) and their own domain lengths (so their own dx, dy
and time steps), sharing what a batch shares (order k = 3..6, system, boundaries, OE off or
Type II, positivity limiter on some Euler batches).  Two steps of the batched context (one launch
per stage over the work list of all instances) must equal, bit for bit, two steps of one context
per instance, and match the oracle run on each instance to the parity bar (relative L-infinity
1e-12).
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
TOL = 1e-12
NBATCH = 10


def _batch(b):
    rng = np.random.default_rng(7000 + b)
    system = ("advection", "burgers", "euler", "euler", "euler")[b % 5]
    k = int(rng.integers(3, 7))
    bcs = ("periodic", "transmissive")
    bc_x, bc_y = bcs[int(rng.integers(2))], bcs[int(rng.integers(2))]
    oe = ("off", "type2")[int(rng.integers(2))]
    pp = system == "euler" and bool(rng.integers(2))
    if pp:
        bc_x = bc_y = "transmissive"
    n = int(rng.integers(3, 7))
    out = []
    for i in range(n):
        nx, ny = int(rng.integers(3, 121)), int(rng.integers(3, 121))
        lx, ly = float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.5, 2.0))
        kw = dict(dim=2, nx=nx, ny=ny, x0=0.0, x1=lx, y0=0.0, y1=ly, k=k, system=system, bc_x=bc_x, bc_y=bc_y,
                  oe=oe, cfl=0.2, pp=pp)
        if system == "advection":
            kw.update(a=(0.8, -0.5))
        seed = 8000 + 16 * b + i
        if system == "euler":
            U0 = fi.four_quadrant(nx, seed, ny=ny) if pp else fi.random_euler_state_2d(nx, ny, seed, amp=0.2)
        else:
            U0 = fi.random_state((1, 3, ny, nx), seed, 0.2, 1.2)
        out.append((kw, U0))
    return out


@pytest.mark.parametrize("b", range(NBATCH))
def test_random_batch_two_steps(b):
    from paper_2609_26194_amd import Fam
    inst = _batch(b)
    log(f"  batch {b}: {len(inst)} instances, " + ", ".join(f"{kw['nx']}x{kw['ny']}" for kw, _ in inst)
        + f"; k={inst[0][0]['k']} {inst[0][0]['system']} {inst[0][0]['bc_x']}/{inst[0][0]['bc_y']} "
        f"oe={inst[0][0]['oe']} pp={inst[0][0]['pp']}")
    pairs = [both_configs(**kw) for kw, _ in inst]
    cfgs = [c for _, c in pairs]
    bat = Fam(cfgs[0], batch=cfgs)
    offs = bat.offsets()
    Ub = torch.zeros(bat.len, dtype=torch.float64, device="cuda")
    for o, (_, U0) in zip(offs, inst):
        Ub[o:o + U0.size] = to_dev(U0).reshape(-1)
    done, _ = bat.run(Ub, 0.0, 2)
    bat.check()
    bat.close()
    assert done == 2
    worst = 0.0
    for i, (o, (kw, U0)) in enumerate(zip(offs, inst)):
        got = Ub[o:o + U0.size].reshape(U0.shape)
        single = Fam(cfgs[i])
        U = to_dev(U0)
        single.run(U, 0.0, 2)
        single.check()
        single.close()
        assert torch.equal(got, U), f"instance {i}: batched and single-context states differ"
        ref, _, steps = S.run(torch.tensor(U0), pairs[i][0], nsteps=2)
        assert steps == 2
        err = rel_linf(got, ref)
        worst = max(worst, err)
        assert err <= TOL, f"instance {i}: rel Linf {err:.2e}"
    log(f"    worst rel Linf {worst:.2e}")
