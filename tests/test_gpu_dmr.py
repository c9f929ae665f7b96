"""Double Mach reflection boundaries (Sec. 4 example) on the GPU against the oracle.

The library applies the example's boundary data in the row loader that every 2D
strip kernel uses (post-shock inflow on the left, copy on the right, on the bottom
the post-shock state for x < 1/6 and a reflecting wall beyond, on the top the
exact moving shock at the stage's time).  The oracle builds the same ghost
cells explicitly (oracle/scheme.py, _pad_dmr) at each RK stage's time and the OE
time.  Coarse meshes of the example's domain [0, 3] x [0, 1] run a few steps
(the top shock moves by about a cell) with the positivity limiter, as in the
paper's run.
"""
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
TOL = 1e-12


def _fam(cfg):
    from paper_2609_26194_amd import Fam
    return Fam(cfg)


@pytest.mark.parametrize("k,nx,ny,nsteps", [(5, 96, 32, 8), (3, 60, 20, 12), (6, 72, 24, 6)])
def test_double_mach_boundaries_match_the_oracle(k, nx, ny, nsteps):
    log(f"double Mach reflection k={k} {nx}x{ny}, {nsteps} steps")
    ora, cfg = both_configs(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=k, system="euler", oe="type2",
                            cfl=0.2, pp=True, dmr=True, bc_x="transmissive", bc_y="transmissive")
    U0 = fi.double_mach(nx, ny)
    ref, t_ref, steps_ref = S.run(torch.tensor(U0), ora, nsteps=nsteps)
    fam = _fam(cfg)
    U = to_dev(U0)
    steps, t = fam.run(U, 0.0, nsteps)
    fam.check()
    assert steps == steps_ref and abs(t - t_ref) <= 1e-14
    err = rel_linf(U, ref)
    log(f"  t = {t:.4e}, rel Linf {err:.3e}")
    assert err <= TOL


def test_double_mach_segment_list_and_fixed_tiles_agree():
    """The boundary rows and columns are handled in the row loader, so any tiling gives the
    same state (bitwise)."""
    nx, ny = 300, 100
    _, cfg = both_configs(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2",
                          cfl=0.2, pp=True, dmr=True)
    U0 = to_dev(fi.double_mach(nx, ny))
    outs = []
    for hs, ho in ((16, 16), (0, 24), (40, 8)):
        fam = _fam(cfg)
        fam.set_tiling(hs, ho)
        U = U0.clone()
        fam.run(U, 0.0, 20)
        fam.check()
        outs.append(U)
        fam.close()
    for U in outs[1:]:
        assert torch.equal(U, outs[0])


def test_double_mach_rejected_where_unsupported():
    from paper_2609_26194_amd import Fam, FamConfig
    from paper_2609_26194_amd.fam import FamError
    with pytest.raises(FamError):
        Fam(FamConfig(dim=2, nx=30, ny=10, system="advection", dmr=True))
    fam = Fam(FamConfig(dim=2, nx=30, ny=10, x1=3.0, system="euler", dmr=True, bc_x="periodic", bc_y="periodic"))
    U = to_dev(fi.double_mach(30, 10))
    with pytest.raises(FamError):
        fam.dbg_recon(U)
    with pytest.raises(FamError):
        fam.adjoint(U, 2, 1e-4, 1)


def test_double_mach_steps_continue_the_clock():
    """The context clock carries the time from one call to the next: the top boundary's
    moving shock is placed at each RK stage's time in every fam_step call and in every
    replay of a captured fam_step, so N eager steps and N replays equal fam_run over N
    steps bit for bit (and the oracle), after fam_set_time(0) brings the clock back."""
    nx, ny, nsteps = 96, 32, 6
    log(f"double Mach reflection {nx}x{ny}: fam_step / graph replays / fam_run over {nsteps} steps")
    ora, cfg = both_configs(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2",
                            cfl=0.2, pp=True, dmr=True)
    U0h = fi.double_mach(nx, ny)
    U0 = to_dev(U0h)
    fam = _fam(cfg)
    Ur = U0.clone()
    steps, t = fam.run(Ur, 0.0, nsteps)
    fam.check()
    assert steps == nsteps
    ref, t_ref, _ = S.run(torch.tensor(U0h), ora, nsteps=nsteps)
    assert abs(t - t_ref) <= 1e-14 and rel_linf(Ur, ref) <= TOL
    # eager steps from the restarted clock
    fam.set_time(0.0)
    Ue = U0.clone()
    for _ in range(nsteps):
        fam.step(Ue)
    torch.cuda.synchronize()
    fam.check()
    assert torch.equal(Ue, Ur)
    # replays of one captured step
    fam.set_time(0.0)
    Ug = U0.clone()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=fam.stream):
        fam.step(Ug)
    torch.cuda.synchronize()
    for _ in range(nsteps):
        g.replay()
    torch.cuda.synchronize()
    fam.check()
    assert torch.equal(Ug, Ur)
    # the clock has reached the run's end time; a run to that time does nothing
    Uz = Ur.clone()
    n0, t0 = fam.run(Uz, t, 0)
    assert n0 == 0 and torch.equal(Uz, Ur) and abs(t0 - t) <= 1e-15
    log(f"  t = {t:.4e}: eager steps and replays equal fam_run bitwise; rel Linf vs oracle {rel_linf(Ur, ref):.2e}")
    del g
    fam.close()
