"""Pins of the oracle's local characteristic-variable reconstruction (the FAM5
alternative timed in Sec. 4.3, Table runtime-main Panel B).

* The eigenvectors: L R = I, and R diag(u_n - c, u_n, u_n + c[, u_n]) L equals the
  flux Jacobian, taken by automatic differentiation of the flux (an independent
  route to the same matrix), in 1D and in both 2D directions.
* Sec. 2.3's remark that the linear reconstruction commutes with a fixed change of
  variables: the characteristic and the conservative stage reconstructions agree
  to rounding for every order, in 1D and 2D, and so do whole steps (with the
  positivity limiter and with the double Mach reflection boundaries).  Where a
  component is identically zero over a region (the momentum ahead of the
  Shu-Osher and double-Mach shocks), the conservative path keeps it exactly zero
  while the transform leaves rounding noise in it, and the Type II coefficient
  gamma_k J / D of that component is then a ratio of two noise-level numbers once
  D passes the guard eps: such runs are compared with OE off, and the
  amplification itself is pinned as a property of the OE (a few steps lift the
  difference far above rounding, OE off keeps it at rounding).
* Sensitivity: the same comparison with a planted mistake (the back-transform
  taken from a neighbouring cell's state) fails by orders of magnitude.
"""
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from oracle.physics import Euler

DT = torch.float64


def _states(dim, n, seed):
    g = torch.Generator().manual_seed(seed)
    rho = 0.2 + 2.0 * torch.rand(n, generator=g, dtype=DT)
    p = 0.05 + 3.0 * torch.rand(n, generator=g, dtype=DT)
    vel = [2.0 * torch.randn(n, generator=g, dtype=DT) for _ in range(dim)]
    E = p / 0.4 + 0.5 * rho * sum(v * v for v in vel)
    return torch.stack([rho] + [rho * v for v in vel] + [E]), rho, p, vel


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_eigenvectors_diagonalise_the_flux_jacobian(dim, d):
    ph = Euler(dim)
    u, rho, p, vel = _states(dim, 12, 3 + dim + d)
    L, R = ph.eigen(u, d)
    I = torch.einsum("ij...,jk...->ik...", L, R)
    assert float((I - torch.eye(dim + 2, dtype=DT)[..., None]).abs().max()) < 1e-12
    c = torch.sqrt(1.4 * p / rho)
    for n in range(u.shape[1]):
        J = torch.autograd.functional.jacobian(lambda x: ph.flux(x, d), u[:, n].clone())
        un = vel[d][n]
        lam = [un - c[n], un, un + c[n]] + ([un] if dim == 2 else [])
        A = R[:, :, n] @ torch.diag(torch.stack(lam)) @ L[:, :, n]
        assert float((A - J).abs().max()) <= 1e-12 * max(1.0, float(J.abs().max()))


def _rel(a, b):
    return float((a - b).abs().max()) / float(b.abs().max())


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("dim", [1, 2])
def test_characteristic_reconstruction_commutes(dim, k):
    if dim == 1:
        cfg = S.Config(dim=1, nx=40, k=k, system="euler", char_vars=True)
        U = torch.tensor(fi.shu_osher(40))
    else:
        cfg = S.Config(dim=2, nx=24, ny=20, k=k, system="euler", char_vars=True)
        U = torch.tensor(fi.four_quadrant(24, seed=5, ny=20))
    Upad = S.pad(U, cfg)
    _, cw = S.reconstruct_stage(Upad, cfg)
    _, cc = S.reconstruct(Upad, cfg)
    assert _rel(cw, cc) < 1e-12


def test_planted_back_transform_mistake_is_caught():
    cfg = S.Config(dim=2, nx=24, ny=20, k=5, system="euler", char_vars=True)
    U = torch.tensor(fi.four_quadrant(24, seed=5, ny=20))
    Upad = S.pad(U, cfg)
    monos, Rm = S.recon_matrix(2, 5)
    St = S.stencil_2d(Upad, 5)
    avg = Upad[:, 0, 1:-1, 1:-1]
    L, _ = cfg.phys.eigen(avg, 0)
    _, Rwrong = cfg.phys.eigen(torch.roll(avg, 1, dims=-1), 0)
    W = torch.einsum("ab...,bi...->ai...", L, St)
    bad = torch.einsum("ca...,ap...->cp...", Rwrong, torch.einsum("pi,ai...->ap...", Rm, W))
    _, cc = S.reconstruct(Upad, cfg)
    assert _rel(bad, cc) > 1e-3


def _case(case):
    if case.startswith("shu_osher"):
        kw = dict(dim=1, nx=200, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive", oe="off")
        U = torch.tensor(fi.shu_osher(200))
    elif case == "smooth_1d":
        kw = dict(dim=1, nx=40, x0=0.0, x1=2.0, k=5, system="euler")
        U = torch.tensor(fi.smooth_euler_1d(40))
    elif case == "four_quadrant_pp":
        kw = dict(dim=2, nx=32, ny=32, k=5, system="euler", pp=True)
        U = torch.tensor(fi.four_quadrant(32, seed=0))
    elif case == "density_waves":
        kw = dict(dim=2, nx=24, ny=24, k=6, system="euler")
        U = torch.tensor(fi.density_waves(24))
    else:
        kw = dict(dim=2, nx=48, ny=16, x0=0.0, x1=3.0, k=5, system="euler", pp=True, dmr=True, oe="off")
        U = torch.tensor(fi.double_mach(48, 16))
    return kw, U


@pytest.mark.parametrize("case", ["shu_osher", "smooth_1d", "four_quadrant_pp", "density_waves", "double_mach"])
def test_characteristic_steps_match_conservative_steps(case):
    kw, U = _case(case)
    a, ta, na = S.run(U.clone(), S.Config(char_vars=True, **kw), nsteps=3)
    b, tb, nb = S.run(U.clone(), S.Config(**kw), nsteps=3)
    assert na == nb and abs(ta - tb) <= 1e-14
    assert _rel(a, b) < 1e-12


def test_type2_oe_amplifies_rounding_in_identically_zero_components():
    kw, U = _case("shu_osher")
    kw["oe"] = "type2"
    a, _, _ = S.run(U.clone(), S.Config(char_vars=True, **kw), nsteps=3)
    b, _, _ = S.run(U.clone(), S.Config(**kw), nsteps=3)
    assert _rel(a, b) > 1e-10


def test_characteristic_variables_need_euler():
    with pytest.raises(ValueError):
        S.Config(dim=1, nx=8, system="burgers", char_vars=True)
