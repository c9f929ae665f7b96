"""Invariants of the oracle's step that the paper fixes or that follow from its definitions.

* OE (Props. 2.1-2.3): cell averages unchanged bit for bit, 0 < delta <= 1, first
  moments damped nonexpansively, no damping on data the reconstruction reproduces.
* Conservation: with face fluxes computed once per face, sum of u^(0) dx dy is
  constant to roundoff on periodic meshes (eq. 11 summed over cells).
* The Cartesian scheme on y-independent data equals the 1D scheme (uniqueness of
  the moment systems: the 1D polynomial satisfies the 2D constraints).
* x <-> y transpose equivariance on square meshes.
* Building blocks: 4-point Gauss exact to degree 7; Rusanov flux consistent.
* The positivity limiter leaves admissible reconstructions untouched and makes
  every flux point admissible.
"""

import numpy as np
import pytest
import torch

import fam_inputs as fi
from oracle import physics
from oracle.physics import NonPhysicalState, gauss4
from oracle.scheme import Config, oe, oe_delta, pad, points_2d, point_values, pp_apply, pp_theta, \
    reconstruct, residual, rk3, run, step


def euler2d(n, **kw):
    base = dict(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="periodic", bc_y="periodic",
                oe="type2", cfl=0.2)
    base.update(kw)
    return Config(**base)


def test_gauss_rule_exact_to_degree_7():
    x, w = gauss4()
    assert abs(sum(w) - 1.0) < 1e-16
    for p in range(8):
        exact_val = 0.0 if p % 2 else (0.5 ** p) / (p + 1)
        assert abs(sum(wi * xi ** p for xi, wi in zip(x, w)) - exact_val) < 1e-16


def test_rusanov_consistent_and_upwind():
    ph = physics.Euler(2)
    u = torch.tensor(fi.random_euler_state_2d(5, 4, 3)[:, 0])
    for d in (0, 1):
        s = physics.max_speed(ph, u, d)
        assert torch.allclose(physics.rusanov(ph, u, u, d, s), ph.flux(u, d), rtol=0, atol=0)
    adv = physics.Advection((1.5, 0.0))
    a, b = torch.rand(1, 7, dtype=torch.float64), torch.rand(1, 7, dtype=torch.float64)
    s = physics.max_speed(adv, a, 0)
    assert torch.allclose(physics.rusanov(adv, a, b, 0, s), 1.5 * a, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_oe_invariants_2d(k):
    cfg = euler2d(24, k=k, bc_x="transmissive", bc_y="transmissive", pp=True)
    U = torch.tensor(fi.four_quadrant(24, 7))
    Un = rk3(U, 2e-3, cfg)
    Us = oe(Un, 2e-3, cfg)
    assert torch.equal(Us[:, 0], Un[:, 0])
    ratio = Us[:, 1:] / torch.where(Un[:, 1:] == 0, torch.ones_like(Un[:, 1:]), Un[:, 1:])
    mask = Un[:, 1:] != 0
    r = ratio[mask]
    assert bool((r > 0).all()) and bool((r <= 1).all())
    assert bool((torch.abs(Us[:, 1:]) <= torch.abs(Un[:, 1:])).all())
    # one common factor per cell for both moments and all components
    mags = torch.abs(Un[:, 1:]).reshape(8, *Un.shape[2:])
    idx = torch.argmax(mags, dim=0, keepdim=True)
    delta = torch.gather(ratio.reshape(8, *Un.shape[2:]), 0, idx)[0]
    err = torch.abs(Us[:, 1:] - delta * Un[:, 1:])
    assert bool((err <= 1e-15 * torch.abs(Un[:, 1:])).all())
    # strong jumps are damped somewhere
    assert float(r.min()) < 0.99


@pytest.mark.parametrize("dim", [1, 2])
def test_oe_delta_is_the_factor_oe_applies(dim):
    """oe_delta returns the per-cell factor that oe multiplies both first moments by."""
    if dim == 2:
        cfg = euler2d(20, bc_x="transmissive", bc_y="transmissive")
        U = torch.tensor(fi.four_quadrant(20, 3))
    else:
        cfg = Config(dim=1, nx=200, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive", oe="type1")
        U = torch.tensor(fi.shu_osher(200))
    d = oe_delta(U, 2e-3, cfg)
    assert d.shape == U.shape[2:]
    assert bool((d > 0).all()) and bool((d <= 1).all()) and float(d.min()) < 0.99
    assert torch.equal(oe(U, 2e-3, cfg)[:, 1:], U[:, 1:] * d)


def test_oe_invariants_1d():
    cfg = Config(dim=1, nx=400, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive",
                 oe="type2")
    U = torch.tensor(fi.shu_osher(400))
    Un = rk3(U, 1e-3, cfg)
    Us = oe(Un, 1e-3, cfg)
    assert torch.equal(Us[:, 0], Un[:, 0])
    assert bool((torch.abs(Us[:, 1]) <= torch.abs(Un[:, 1])).all())
    d = Us[:, 1] / torch.where(Un[:, 1] == 0, torch.ones_like(Un[:, 1]), Un[:, 1])
    assert float(d.min()) < 0.9  # the shock is damped


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_oe_no_damping_on_reproduced_polynomials(k):
    """Prop. 2.3(ii) limit case: polynomial data of degree < k has zero jumps."""
    n = 16
    coeffs = np.random.default_rng(k).uniform(-1, 1, 8)

    def f(X, Y):
        P = sum(coeffs[i] * X ** a * Y ** (d - a)
                for i, (d, a) in enumerate([(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (2, 0)]))
        P = P + (coeffs[6] * X ** 2 * Y if k > 3 else 0.0)
        return (3.0 + P)[None]
    U = torch.tensor(fi.moments_2d(f, -1.0, 1.0, -1.0, 1.0, n, n))
    cfg = Config(dim=2, nx=n, ny=n, x0=-1, x1=1, y0=-1, y1=1, k=k, system="advection",
                 a=(1.0, 0.5), bc_x="transmissive", bc_y="transmissive", oe="type2")
    Us = oe(U, 0.01, cfg)
    inner = (slice(None), slice(1, 3), slice(3, -3), slice(3, -3))
    rel = torch.abs(Us[inner] - U[inner]) / torch.abs(U[inner]).clamp(min=1e-300)
    assert float(rel.max()) < 1e-11
    # zero data takes the eps branch: no damping at all
    Z = torch.zeros_like(U)
    Z[:, 1:] = 0.0
    assert torch.equal(oe(Z, 0.01, cfg), Z)
    # Type I on constant data: D_Omega = 0 < eps_Omega
    C = torch.zeros_like(U)
    C[:, 0] = 2.5
    C[:, 1] = 0.1
    cfg1 = Config(dim=2, nx=n, ny=n, k=k, system="advection", oe="type1")
    assert torch.equal(oe(C, 0.01, cfg1), C)


@pytest.mark.parametrize("oe_type", ["off", "type1", "type2"])
def test_conservation_periodic_2d(oe_type):
    cfg = euler2d(20, oe=oe_type)
    U = torch.tensor(fi.random_euler_state_2d(20, 20, 11, amp=0.2))
    tot0 = U[:, 0].sum(dim=(1, 2))
    U, _, _ = run(U, cfg, nsteps=3)
    tot = U[:, 0].sum(dim=(1, 2))
    assert torch.allclose(tot, tot0, rtol=1e-14, atol=1e-13)


def test_conservation_periodic_1d():
    cfg = Config(dim=1, nx=64, k=6, system="euler", oe="type2", x0=0.0, x1=2.0)
    U = torch.tensor(fi.smooth_euler_1d(64))
    tot0 = U[:, 0].sum(dim=1)
    U, _, _ = run(U, cfg, nsteps=5)
    assert torch.allclose(U[:, 0].sum(dim=1), tot0, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("oe_type", ["off", "type1"])
def test_2d_reduces_to_1d_on_y_independent_data(k, oe_type):
    n, ny = 40, 6
    U1 = torch.tensor(fi.shu_osher(n))
    U1[1] *= 0.3  # subsonic, to keep it mild
    # the default gamma_k differs between 1D and 2D for k = 5, 6: use one value
    cfg1 = Config(dim=1, nx=n, x0=-5.0, x1=5.0, k=k, system="euler", bc_x="transmissive",
                  oe=oe_type, oe_gamma_k=20.0)
    cfg2 = Config(dim=2, nx=n, ny=ny, x0=-5.0, x1=5.0, y0=0.0, y1=1.0, k=k, system="euler",
                  bc_x="transmissive", bc_y="periodic", oe=oe_type, oe_gamma_k=20.0)
    U2 = torch.zeros(4, 3, ny, n, dtype=torch.float64)
    for c2, c1 in ((0, 0), (1, 1), (3, 2)):
        U2[c2, 0] = U1[c1, 0]
        U2[c2, 1] = U1[c1, 1]
    dt = 2e-3
    A, _, _ = run(U1, cfg1, nsteps=3, dt=dt)
    B, _, _ = run(U2, cfg2, nsteps=3, dt=dt)
    for c2, c1 in ((0, 0), (1, 1), (3, 2)):
        for r in (0, 1):
            diff = torch.abs(B[c2, r] - A[c1, r][None, :]).max()
            assert float(diff) < 1e-12 * float(torch.abs(A[c1, 0]).max())
        assert float(torch.abs(B[c2, 2]).max()) < 1e-14
    assert float(torch.abs(B[2]).max()) < 1e-14


def _transpose(U):
    T = U.transpose(-1, -2).clone()
    T = T[[0, 2, 1, 3]]          # swap momentum components
    return T[:, [0, 2, 1]]       # swap x- and y-moments


@pytest.mark.parametrize("oe_type", ["off", "type2"])
def test_transpose_equivariance(oe_type):
    cfg = euler2d(18, oe=oe_type, bc_x="transmissive", bc_y="transmissive", pp=True)
    U = torch.tensor(fi.four_quadrant(18, 5, split=(0.4, 0.6)))
    A, _ = step(U, cfg, 1e-3)
    B, _ = step(_transpose(U), cfg, 1e-3)
    assert float(torch.abs(_transpose(B) - A).max()) < 1e-13


def test_pp_limiter_inactive_on_admissible_data():
    cfg = euler2d(16)
    U = torch.tensor(fi.random_euler_state_2d(16, 16, 2, amp=0.1))
    cfg_pp = euler2d(16, pp=True)
    assert torch.equal(residual(U, cfg), residual(U, cfg_pp))


def test_pp_limiter_makes_flux_points_admissible():
    n = 24
    cfg = euler2d(n, bc_x="transmissive", bc_y="transmissive", pp=True)
    U = torch.tensor(fi.four_quadrant(n, 0))
    Upad = pad(U, cfg)
    monos, coef = reconstruct(Upad, cfg)
    vals = point_values(monos, coef, points_2d())
    ph = cfg.phys
    assert float(ph.pressure(vals).min()) < 0      # unlimited: negative pressure
    avg = Upad[:, 0, 1:-1, 1:-1]
    th1, th2 = pp_theta(vals, avg, ph)
    lim = pp_apply(vals, avg, th1, th2)
    assert float(lim[0].min()) > 0 and float(ph.pressure(lim).min()) > 0
    assert float(th2.min()) < 1 and float(th2.max()) == 1.0
    # tightness: where the pressure scaling is active, the smallest limited pressure
    # over the 32 points sits at the floor eps <= 1e-13 (up to rounding), so the
    # scaling is the largest admissible one, not merely an admissible one
    active = th2 < 1.0
    pmin = ph.pressure(lim).min(dim=0).values
    assert float(pmin[active].max()) < 1e-10
    # the limited reconstruction keeps the cell average (volume-point quadrature)
    _, w = gauss4()
    W = torch.tensor([w[q % 4] * w[q // 4] for q in range(16)], dtype=torch.float64)
    qavg = torch.einsum("q,cq...->c...", W, lim[:, 16:])
    assert torch.allclose(qavg, avg, rtol=1e-13, atol=1e-13)


def test_nonphysical_state_is_reported():
    U = torch.tensor(fi.random_euler_state_2d(16, 16, 2))
    U[0, 0, 3, 4] = -0.5  # negative density in one cell average
    with pytest.raises(NonPhysicalState):
        step(U, euler2d(16))
    U = torch.tensor(fi.random_euler_state_2d(16, 16, 2))
    U[3, 0, 5, 5] = 0.01  # energy below kinetic: negative pressure in one cell average
    with pytest.raises(NonPhysicalState):
        step(U, euler2d(16, pp=True))


@pytest.mark.parametrize("dim", [1, 2])
def test_uniform_state_is_a_fixed_point_bit_for_bit(dim):
    """On a uniform periodic flow every cell computes the same values, so the average
    residual R^(0) is exactly zero and every RK stage must return the averages of U^n
    bit for bit: true when the convex combination of eq. 12 is formed as
    L + c (U^n - L), not with the weights 1/3 and 2/3 rounded separately (their sum is
    1 - 2^-54, and a generic value drifts).  (The first moments move at rounding level:
    the quadrature weights do not sum to one exactly.)"""
    rng = np.random.default_rng(5 + dim)
    for _ in range(4):
        rho, p = rng.uniform(0.2, 3.0), rng.uniform(0.1, 4.0)
        vel = rng.uniform(-1.5, 1.5, dim)
        E = p / 0.4 + 0.5 * rho * float(np.sum(vel * vel))
        vals = [rho] + list(rho * vel) + [E]
        if dim == 1:
            cfg = Config(dim=1, nx=12, k=5, system="euler", oe="type2")
            U = torch.zeros(3, 2, 12, dtype=torch.float64)
        else:
            cfg = euler2d(10)
            U = torch.zeros(4, 3, 10, 10, dtype=torch.float64)
        for c, v in enumerate(vals):
            U[c, 0] = v
        U0 = U.clone()
        for _ in range(20):
            U, _ = step(U, cfg)
        assert torch.equal(U[:, 0], U0[:, 0])
