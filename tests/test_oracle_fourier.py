"""Pins of the oracle's semi-discrete operator and RK3 against the Fourier analysis of Sec. 3.

* Table tab_Dk: the operator for u_t + u_x = 0 (Rusanov = upwind here), applied to
  unit moment vectors on a periodic mesh, must reproduce the printed 2x2 blocks
  D_{-2..1} (eq. linear-semi).
* The spurious eigenvalue at xi -> 0 (appendix of full asymptotic expansions):
  zeta_2 dx -> -6, -60/11, -205/54, -35/9.
* The physical-mode error zeta_1 + i omega has the printed leading term.
* Prop. 3.4: sampled admissible CFL numbers 0.40, 0.44, 0.58, 0.56 (truncated).
* Closed form of the fully discrete linear backbone: U^n = G(xi)^n u_ex per Fourier
  mode (eq. Gmatrix2 with the printed D matrices and the printed exact moment
  vector u_ex) must equal the oracle's own time stepping with OE off.
"""
import math

import numpy as np
import pytest
import torch

import fam_inputs as fi
from golden_util import parse_matrices
from oracle.scheme import Config, residual, run

GOLD_D = parse_matrices("fourier_D_matrices.txt")
ZETA2 = {3: -6.0, 4: -60.0 / 11.0, 5: -205.0 / 54.0, 6: -35.0 / 9.0}


def oracle_D(k, n=16):
    """D_l (l = -2..1) extracted from the oracle's R(U) for u_t + u_x = 0."""
    cfg = Config(dim=1, nx=n, k=k, system="advection", a=(1.0, 0.0), oe="off",
                 x0=0.0, x1=float(n))  # dx = 1
    j = n // 2
    D = np.zeros((4, 2, 2))
    for r in range(2):
        U = torch.zeros(1, 2, n, dtype=torch.float64)
        U[0, r, j] = 1.0
        R = residual(U, cfg)[0].numpy()            # [2, n]
        for li, ell in enumerate((-2, -1, 0, 1)):
            D[li, :, r] = R[:, j - ell] * cfg.dx
        # nothing outside the 4-cell stencil
        mask = np.ones(n, bool)
        mask[[j + 2, j + 1, j, j - 1]] = False
        assert np.all(R[:, mask] == 0.0)
    return D


def symbol(D, xi):
    """G_hat(xi) = sum_l D_l exp(i l xi) (eq. Gmatrix times dx); xi may be an array."""
    xi = np.asarray(xi, dtype=np.float64)[..., None, None]
    return sum(D[li] * np.exp(1j * ell * xi) for li, ell in enumerate((-2, -1, 0, 1)))


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_operator_reproduces_printed_D_matrices(k):
    D = oracle_D(k)
    gold = np.array([[[float(v) for v in row] for row in M] for M in GOLD_D[f"k{k}"]])
    np.testing.assert_allclose(D, gold, rtol=0, atol=2e-14)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_spurious_eigenvalue_limit(k):
    ev = np.linalg.eigvals(symbol(oracle_D(k), 0.0))
    ev = ev[np.argsort(np.abs(ev))]
    assert abs(ev[0]) < 1e-13
    assert abs(ev[1] - ZETA2[k]) < 1e-12


# leading terms of zeta_1 + i omega (omega = 1): c * dx^(k+1), complex c
LEAD = {3: (-1j / 720.0, 4), 4: (-11.0 / 7200.0, 5), 5: (1j / 114800.0, 6), 6: (-1.0 / 19600.0, 7)}


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_physical_mode_leading_error(k):
    D = oracle_D(k)
    c, p = LEAD[k]
    ratios = []
    for dx in (0.4, 0.2, 0.1):
        ev = np.linalg.eigvals(symbol(D, dx)) / dx
        z1 = ev[np.argmin(np.abs(ev + 1j))]
        ratios.append((z1 + 1j) / (c * dx ** p))
    # the component along the printed coefficient -> 1; the orthogonal part is the
    # next (O(dx^{k+2})) term and shrinks linearly with dx
    assert abs(ratios[-1].real - 1) < 0.1
    assert abs(ratios[-1].imag) < 0.6 * abs(ratios[1].imag) + 1e-3
    assert abs(ratios[1].imag) < 0.6 * abs(ratios[0].imag) + 1e-3


def _rk3_amp(Z):
    I = np.eye(2)
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6


def _spectral_radius_max(D, C, xis):
    Z = C * symbol(D, xis)
    G = _rk3_amp(Z)
    tr = G[:, 0, 0] + G[:, 1, 1]
    det = G[:, 0, 0] * G[:, 1, 1] - G[:, 0, 1] * G[:, 1, 0]
    disc = np.sqrt(tr * tr - 4 * det)
    return np.max(np.maximum(np.abs((tr + disc) / 2), np.abs((tr - disc) / 2)))


@pytest.mark.parametrize("k,printed", [(3, 0.40), (4, 0.44), (5, 0.58), (6, 0.56)])
def test_sampled_cfl(k, printed):
    """Prop. 3.4: largest C with rho(G) <= 1 on 10^4 uniform samples of [0, 2 pi]."""
    D = oracle_D(k)
    xis = np.linspace(0.0, 2 * math.pi, 10000)
    lo, hi = 0.05, 1.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if _spectral_radius_max(D, mid, xis) <= 1.0 + 1e-12:
            lo = mid
        else:
            hi = mid
    assert math.floor(lo * 100) / 100 == pytest.approx(printed)


def _u_ex(xi):
    """Printed exact moment vector of exp(i omega x) per cell (Sec. 3)."""
    return np.array([2 * np.sin(xi / 2) / xi,
                     1j * (2 * np.sin(xi / 2) - xi * np.cos(xi / 2)) / xi ** 2])


def closed_form_sine_advection(k, n, nsteps, C):
    """U^n for u0 = sin x + cos(3x)/2 from G(xi)^n with the printed D matrices."""
    D = np.array([[[float(v) for v in row] for row in M] for M in GOLD_D[f"k{k}"]])
    dx = 2 * math.pi / n
    xc = (np.arange(n) + 0.5) * dx
    out = np.zeros((2, n))
    for omega, amp, shift in ((1, 1.0, -1j), (3, 0.5, 1.0)):
        # sin x = Re(-i e^{ix}); cos 3x = Re(e^{3ix})
        xi = omega * dx
        G = _rk3_amp(C * symbol(D, xi))
        v = np.linalg.matrix_power(G, nsteps) @ _u_ex(xi)
        out += amp * np.real(shift * np.outer(v, np.exp(1j * omega * xc)))
    return out


@pytest.mark.parametrize("k", [3, 5])
def test_closed_form_evolution_matches_oracle_steps(k):
    """Sine advection with OE off: oracle steps == G(xi)^n u_ex to ~1e-13."""
    n, C = 64, 0.2
    nsteps = 5 * n  # t = 2 pi with dt = 0.2 dx
    cfg = Config(dim=1, nx=n, k=k, system="advection", oe="off", x0=0.0, x1=2 * math.pi)
    U0 = torch.tensor(fi.sine_advection(n))
    dt = 2 * math.pi / nsteps
    assert abs(dt - C * cfg.dx) < 1e-15
    U, _, steps = run(U0, cfg, nsteps=nsteps, dt=dt)
    ref = closed_form_sine_advection(k, n, nsteps, C)
    assert np.max(np.abs(U[0].numpy() - ref)) < 5e-13
