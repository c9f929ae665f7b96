"""Pins of the oracle's two-dimensional semi-discrete operator (eq. 11) against the
mathematics, independent of the scheme's own formulas.

* Polynomial exactness (Prop. 2.5(ii) with the 4-point Gauss rule): for linear
  advection u_t + a . grad u = 0 and data that are the exact cell moments of a
  polynomial of total degree <= k - 1, the reconstruction reproduces the polynomial
  on every cell whose stencil lies in the mesh, the two traces at a face agree (so
  the Rusanov flux is a . n u exactly), and the 4-point rule integrates every face
  and volume integrand exactly (degree <= k - 1 <= 7 per direction).  So all three
  components of R(U) must equal the exact moments of -a . grad u, which this test
  computes in rational arithmetic (fractions.Fraction), without the oracle's
  moment routines.  The polynomial has mixed terms, so the cross-moment terms of
  eq. 11 (the y-face flux weighted by xi in the x-moment equation and the x-face
  flux weighted by eta in the y-moment equation) are nonzero and enter the check;
  a flipped sign or a swapped direction in either of them fails it (planted below,
  in a copy of the operator built here from the oracle's own point values).
* Consistency of the Euler operator: on a smooth periodic state R(U) converges to
  the exact moments of -div f(u), with the divergence taken by automatic
  differentiation of a flux written out here from the conservation law, and
  10-point Gauss quadrature of the moments.
* The Euler wave speed that sets the time step, the Rusanov alpha and the OE beta
  is the spectral radius of the flux Jacobian in that direction: compared with the
  largest eigenvalue modulus of the Jacobian taken by automatic differentiation.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import physics
from oracle.scheme import Config, pad, point_values, points_2d, reconstruct, residual

DT = torch.float64
A_VEL = (0.7, -1.3)


def _int_power(n):
    """Exact integral of xi^n over [-1/2, 1/2]."""
    return Fraction(0) if n % 2 else Fraction(1, (n + 1) * 2 ** n)


def _cell_integral_1d(a, centre, h, p):
    """Exact value of the integral over xi in [-1/2, 1/2] of (centre + h xi)^a xi^p."""
    return sum(Fraction(math.comb(a, m)) * centre ** (a - m) * h ** m * _int_power(m + p) for m in range(a + 1))


def _moments(poly, xc, yc, hx, hy):
    """The three scaled moments (average, x-moment, y-moment) of sum c_ab x^a y^b on a cell."""
    out = []
    for p, q in ((0, 0), (1, 0), (0, 1)):
        out.append(sum(c * _cell_integral_1d(a, xc, hx, p) * _cell_integral_1d(b, yc, hy, q)
                       for (a, b), c in poly.items()))
    return out


def _random_poly(deg, seed):
    rng = random.Random(seed)
    return {(a, b): Fraction(rng.randint(-40, 40), rng.randint(1, 16))
            for a in range(deg + 1) for b in range(deg + 1 - a)}


def _advection_rate(poly):
    """The polynomial -a . grad u (exact time derivative under linear advection)."""
    ax, ay = (Fraction(v).limit_denominator(1000) for v in A_VEL)
    out = {}
    for (a, b), c in poly.items():
        if a > 0:
            out[(a - 1, b)] = out.get((a - 1, b), Fraction(0)) - ax * a * c
        if b > 0:
            out[(a, b - 1)] = out.get((a, b - 1), Fraction(0)) - ay * b * c
    return out


NX, NY = 16, 14
MARGIN = 3


def _mesh_moments(poly):
    hx, hy = Fraction(1, NX), Fraction(1, NY)
    M = np.zeros((3, NY, NX), dtype=object)
    for j in range(NY):
        for i in range(NX):
            xc, yc = (Fraction(2 * i + 1, 2 * NX), Fraction(2 * j + 1, 2 * NY))
            M[:, j, i] = _moments(poly, xc, yc, hx, hy)
    return M


def _cfg(k):
    return Config(dim=2, nx=NX, ny=NY, x0=0.0, x1=1.0, y0=0.0, y1=1.0, k=k, system="advection", a=A_VEL,
                  bc_x="transmissive", bc_y="transmissive", oe="off")


def _polynomial_case(k, seed):
    poly = _random_poly(k - 1, seed)
    U = torch.tensor(_mesh_moments(poly).astype(float), dtype=DT)[None]        # [1, 3, NY, NX]
    want = _mesh_moments(_advection_rate(poly)).astype(float)
    return U, want


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_residual_2d_exact_on_polynomials(k):
    """R(U) equals the exact moment derivatives on data of total degree <= k - 1."""
    for seed in (11 * k, 11 * k + 1):
        U, want = _polynomial_case(k, seed)
        R = residual(U, _cfg(k))[0].numpy()
        inner = (slice(None), slice(MARGIN, NY - MARGIN), slice(MARGIN, NX - MARGIN))
        scale = np.abs(want[inner]).max()
        err = np.abs(R[inner] - want[inner]).max()
        assert err <= 1e-12 * scale, (k, seed, err, scale)
        # each component is active (the moment rates are O(h) against the averages' rates), so
        # each is checked well above the tolerance
        for r in range(3):
            assert np.abs(want[r][inner[1:]]).max() > 1e-4 * scale
        # the x- and y-moment rates need the cross terms: without the y-face flux weighted by xi
        # in the x-moment equation (and the x-face flux weighted by eta in the y-moment equation)
        # the exact values are not reached
        assert np.abs(_cross_free(U, _cfg(k), (0.0, 0.0))[inner] - want[inner]).max() > 1e-6 * scale


def _cross_free(U, cfg, flip=(1.0, 1.0)):
    """A copy of eq. 11's x- and y-moment residuals built from the oracle's point values,
    with the cross terms scaled by flip = (x-moment factor, y-moment factor); flip = (1, 1)
    keeps them, (0, 0) drops them, (-1, -1) flips their signs."""
    nodes, weights = physics.gauss4()
    monos, coef = reconstruct(pad(U, cfg), cfg)
    vals = point_values(monos, coef, points_2d())[0]                   # [32, NY+2, NX+2]
    ax, ay = A_VEL
    right, left, top, bot = vals[0:4, 1:-1, :], vals[4:8, 1:-1, :], vals[8:12, :, 1:-1], vals[12:16, :, 1:-1]
    F = [ax * torch.where(torch.tensor(ax >= 0), right[g, :, :-1], left[g, :, 1:]) for g in range(4)]
    G = [ay * torch.where(torch.tensor(ay >= 0), top[g, :-1, :], bot[g, 1:, :]) for g in range(4)]
    Fbar = sum(weights[g] * F[g] for g in range(4))
    Ftil = sum(weights[g] * nodes[g] * F[g] for g in range(4))
    Gbar = sum(weights[g] * G[g] for g in range(4))
    Gtil = sum(weights[g] * nodes[g] * G[g] for g in range(4))
    vol = vals[16:32, 1:-1, 1:-1]
    V1 = sum(weights[q % 4] * weights[q // 4] * ax * vol[q] for q in range(16))
    V2 = sum(weights[q % 4] * weights[q // 4] * ay * vol[q] for q in range(16))
    dx, dy = cfg.dx, cfg.dy
    R0 = -(Fbar[:, 1:] - Fbar[:, :-1]) / dx - (Gbar[1:] - Gbar[:-1]) / dy
    R1 = V1 / dx - (Fbar[:, 1:] + Fbar[:, :-1]) / (2 * dx) - flip[0] * (Gtil[1:] - Gtil[:-1]) / dy
    R2 = V2 / dy - (Gbar[1:] + Gbar[:-1]) / (2 * dy) - flip[1] * (Ftil[:, 1:] - Ftil[:, :-1]) / dx
    return torch.stack([R0, R1, R2]).numpy()


@pytest.mark.parametrize("flip", [(-1.0, 1.0), (1.0, -1.0), (0.0, 1.0), (1.0, 0.0)])
def test_planted_cross_term_mistakes_fail_the_pin(flip):
    """The pin's sensitivity: the same exactness check on a copy of the operator with one
    cross term's sign flipped or dropped fails, while the unaltered copy passes."""
    k = 5
    U, want = _polynomial_case(k, 7)
    inner = (slice(None), slice(MARGIN, NY - MARGIN), slice(MARGIN, NX - MARGIN))
    scale = np.abs(want[inner]).max()
    assert np.abs(_cross_free(U, _cfg(k))[inner] - want[inner]).max() <= 1e-12 * scale
    assert np.abs(_cross_free(U, _cfg(k), flip)[inner] - want[inner]).max() > 1e-6 * scale


# ----------------------------------------------------------------------------
# Euler: consistency with -div f, and the spectral radius
# ----------------------------------------------------------------------------
GAMMA = 1.4


def _primitive(x, y):
    tp = 2.0 * math.pi
    rho = 1.0 + 0.2 * torch.sin(tp * (x + 2.0 * y))
    u = 0.5 + 0.1 * torch.cos(tp * y)
    v = -0.3 + 0.1 * torch.sin(tp * x)
    p = 1.0 + 0.1 * torch.cos(tp * (x - y))
    return rho, u, v, p


def _conserved(x, y):
    rho, u, v, p = _primitive(x, y)
    return torch.stack([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def _flux_from_primitives(x, y):
    """(f1, f2) of the 2D Euler equations written from the primitive variables."""
    rho, u, v, p = _primitive(x, y)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    f1 = torch.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
    f2 = torch.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])
    return f1, f2


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * x, 0.5 * w


def _grid(n, xi):
    """Quadrature points of every cell: X, Y of shape [j, i, b, a] (point (xi_a, xi_b) of cell (i, j))."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X = c[None, :, None, None] + h * xi[None, None, None, :]
    Y = c[:, None, None, None] + h * xi[None, None, :, None]
    X, Y = np.broadcast_arrays(X, Y)
    return torch.tensor(np.array(X), dtype=DT), torch.tensor(np.array(Y), dtype=DT)


def _cell_moments(q, w, xi):
    """Average, x- and y-moments over each cell of point values q[..., j, i, b, a]."""
    W = torch.tensor(np.outer(w, w), dtype=DT)
    XI = torch.tensor(xi, dtype=DT)
    return torch.stack([(q * W).sum(dim=(-2, -1)), (q * W * XI[None, :]).sum(dim=(-2, -1)),
                        (q * W * XI[:, None]).sum(dim=(-2, -1))], dim=1)


def _exact_rates(n):
    """Moments of -div f(u(x, y)) on an n x n periodic mesh of [0, 1]^2: divergence by
    automatic differentiation, moments by 10-point Gauss quadrature per direction."""
    xi, w = _gauss(10)
    X, Y = _grid(n, xi)
    X.requires_grad_(True)
    Y.requires_grad_(True)
    f1, f2 = _flux_from_primitives(X, Y)
    div = []
    for c in range(4):
        gx, = torch.autograd.grad(f1[c].sum(), X, retain_graph=True)
        gy, = torch.autograd.grad(f2[c].sum(), Y, retain_graph=True)
        div.append(-(gx + gy).detach())
    return _cell_moments(torch.stack(div), w, xi)           # [4, 3, n, n]


def _exact_state(n):
    xi, w = _gauss(10)
    X, Y = _grid(n, xi)
    return _cell_moments(_conserved(X, Y), w, xi)


@pytest.mark.parametrize("k", [5, 6])
def test_euler_residual_converges_to_the_divergence(k):
    """Each moment's residual approaches the exact rate, relative to that moment's own
    scale: the averages at order ~k, the first moments at order ~k - 1 (the Rusanov
    term's O(h^k) jump divided by h; 4.5-5.7 measured from 12 to 24 cells).  A wrong
    flux component or cross term leaves an O(1) relative error."""
    errs = []
    for n in (12, 24):
        cfg = Config(dim=2, nx=n, ny=n, k=k, system="euler", oe="off")
        R = residual(_exact_state(n), cfg)
        want = _exact_rates(n)
        errs.append([float((R[:, r] - want[:, r]).abs().max() / want[:, r].abs().max()) for r in range(3)])
    for r in range(3):
        order = math.log2(errs[0][r] / errs[1][r])
        assert errs[1][r] < 1e-3 and order > (k - 0.5 if r == 0 else k - 2), (k, r, errs, order)


@pytest.mark.parametrize("dim,d", [(1, 0), (2, 0), (2, 1)])
def test_euler_speed_is_the_spectral_radius_of_the_flux_jacobian(dim, d):
    ph = physics.Euler(dim)
    g = torch.Generator().manual_seed(40 + dim + d)
    n = 16
    rho = 0.1 + 3.0 * torch.rand(n, generator=g, dtype=DT)
    p = 0.01 + 5.0 * torch.rand(n, generator=g, dtype=DT)
    vel = [3.0 * torch.randn(n, generator=g, dtype=DT) for _ in range(dim)]
    u = torch.stack([rho] + [rho * v for v in vel] + [p / 0.4 + 0.5 * rho * sum(v * v for v in vel)])
    s = ph.speed(u, d)
    for i in range(n):
        J = torch.autograd.functional.jacobian(lambda q: ph.flux(q, d), u[:, i].clone())
        lam = np.abs(np.linalg.eigvals(J.numpy())).max()
        assert abs(float(s[i]) - lam) <= 1e-12 * lam, (i, float(s[i]), lam)
