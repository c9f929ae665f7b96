"""Edge cases of the HIP path: the smallest meshes, degenerate states, and a mesh
whose state planes exceed 2^31 values (64-bit indexing), checked at every cell.

Large mesh: a state that is periodic with a small period P stays periodic with
that period under the scheme (every cell sees the same stencil values as its
image in the P x P problem, and the global wave speeds are the same maxima), so
the full-size result must equal the P x P result tiled, cell for cell.  The P x P
result is the oracle's (relative L-infinity <= 1e-12) and the library's own
(bitwise).
"""
import numpy as np
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


@pytest.mark.parametrize("nx,ny", [(3, 3), (3, 70), (70, 3), (4, 5)])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("k", [3, 5])
def test_smallest_meshes(nx, ny, bc, k):
    log(f"smallest mesh {nx}x{ny} bc={bc} k={k}: 3 steps")
    ora, cfg = both_configs(dim=2, nx=nx, ny=ny, k=k, system="euler", bc_x=bc, bc_y=bc, oe="type2", cfl=0.2)
    U0 = fi.random_euler_state_2d(nx, ny, 21, amp=0.1)
    ref, _, _ = S.run(torch.tensor(U0), ora, nsteps=3)
    fam = _fam(cfg)
    U = to_dev(U0)
    fam.run(U, 0.0, 3)
    fam.check()
    err = rel_linf(U, ref)
    log(f"  rel Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("k", [3, 6])
def test_smallest_1d_mesh(k):
    ora, cfg = both_configs(dim=1, nx=3, k=k, system="euler", bc_x="periodic", oe="type2", cfl=0.2)
    U0 = fi.smooth_euler_1d(3)
    ref, _, _ = S.run(torch.tensor(U0), ora, nsteps=3)
    fam = _fam(cfg)
    U = to_dev(U0)
    fam.run(U, 0.0, 3)
    assert rel_linf(U, ref) <= TOL


@pytest.mark.parametrize("oe", ["type1", "type2", "off"])
def test_uniform_flow_is_a_fixed_point(oe):
    """A uniform state has no jumps and a zero residual (up to the rounding of the
    quadratures); the OE leaves it unchanged (Type II: D < eps is not met, sigma = 0
    from zero jumps; Type I: D_Omega = 0 < eps)."""
    n = 50
    ora, cfg = both_configs(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="periodic", bc_y="periodic",
                            oe=oe, cfl=0.2)
    U0 = np.zeros((4, 3, n, n))
    U0[:, 0] = fi.euler_conservative(np.full((n, n), 1.3), np.full((n, n), 0.4), np.full((n, n), 0.9),
                                     np.full((n, n), -0.7))
    fam = _fam(cfg)
    U = to_dev(U0)
    fam.run(U, 0.0, 5)
    fam.check()
    dev = float((U - to_dev(U0)).abs().max())
    log(f"  uniform flow, oe={oe}: max deviation after 5 steps {dev:.3e}")
    assert dev <= 1e-13
    ref, _, _ = S.run(torch.tensor(U0), ora, nsteps=5)
    assert rel_linf(U, ref) <= TOL


def test_state_planes_beyond_2_31_values_tiled_periodic():
    """16384 x 16384 periodic mesh (each of the 12 planes holds 2^28 values, the
    state 3.2e9), data tiled from a 64 x 64 random state: two steps match the
    64 x 64 run at every cell."""
    P, N, nsteps = 64, 16384, 2
    log(f"tiled periodic {N}x{N} from a {P}x{P} pattern, {nsteps} steps")
    ora_s, cfg_s = both_configs(dim=2, nx=P, ny=P, k=5, system="euler", bc_x="periodic", bc_y="periodic",
                                oe="type2", cfl=0.2, x1=P / N, y1=P / N)
    _, cfg_l = both_configs(dim=2, nx=N, ny=N, k=5, system="euler", bc_x="periodic", bc_y="periodic",
                            oe="type2", cfl=0.2)
    U0 = fi.random_euler_state_2d(P, P, 5, amp=0.1)
    ref, _, _ = S.run(torch.tensor(U0), ora_s, nsteps=nsteps)
    small = _fam(cfg_s)
    Us = to_dev(U0)
    ns, ts = small.run(Us, 0.0, nsteps)
    assert rel_linf(Us, ref) <= TOL
    small.close()
    big = _fam(cfg_l)
    Ub = to_dev(U0).repeat(1, 1, N // P, N // P).contiguous()
    nb, tb = big.run(Ub, 0.0, nsteps)
    big.check()
    assert nb == ns and tb == ts
    # every cell against its image in the small run (bitwise)
    view = Ub.view(4, 3, N // P, P, N // P, P)
    same = torch.equal(view, Us.view(4, 3, 1, P, 1, P).expand_as(view))
    log(f"  bitwise equal to the tiled {P}x{P} result: {same}")
    assert same
    big.close()


@pytest.mark.parametrize("nx,ny", [(3, 3), (70, 3), (3, 70), (125, 9)])
@pytest.mark.parametrize("stage_H", [None, 0])
def test_limiter_on_small_meshes(nx, ny, stage_H):
    """The positivity limiter with the default tiling and with the cost-partitioned segment
    list on meshes smaller than a tile; four-quadrant data whose jumps trip the limiter."""
    log(f"limiter {nx}x{ny}, stage tiling {'default' if stage_H is None else 'segment list'}")
    ora, cfg = both_configs(dim=2, nx=nx, ny=ny, k=5, system="euler", bc_x="transmissive", bc_y="periodic",
                            oe="type2", cfl=0.2, pp=True)
    U0 = fi.four_quadrant(nx, 3, ny=ny) if nx % 2 == 0 and ny % 2 == 0 else fi.random_euler_state_2d(nx, ny, 8, amp=0.6)
    ref, _, _ = S.run(torch.tensor(U0), ora, nsteps=4)
    fam = _fam(cfg)
    if stage_H is not None:
        fam.set_tiling(stage_H, min(8, ny))
    U = to_dev(U0)
    fam.run(U, 0.0, 4)
    fam.check()
    err = rel_linf(U, ref)
    log(f"  rel Linf {err:.3e}")
    assert err <= TOL
