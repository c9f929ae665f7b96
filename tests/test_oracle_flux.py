"""The oracle's Euler flux pinned by physics it must obey (Sec. 2.3: the compressible Euler
equations with the ideal-gas pressure), not by retyping it:

* Rankine-Hugoniot conditions of two exact shocks whose states are fixed independently of the
  oracle: the 1D Mach 3 shock into gas at rest (the jump computed here from the normal-shock
  relations) and the double Mach reflection's 60-degree shock of normal speed 10 (its states as
  published for that example; the shock normal is oblique, so both flux directions enter);
* the eigenvalues of the flux Jacobian (by automatic differentiation of the oracle's flux) are
  u_n - c, u_n (twice in 2D) and u_n + c with the textbook sound speed c = sqrt(gamma p / rho);
* rotation: the y-flux of a state equals the rotated x-flux of the rotated state;
* each planted mistake (pressure dropped from the energy flux, from the momentum flux, the
  velocity of the wrong direction, a wrong (gamma - 1)) fails at least one of the checks.
"""
import math

import numpy as np
import pytest
import torch

from oracle.physics import Euler

G = 1.4


def _flux_n(phys, u, n):
    """Normal flux n_x f_1 + n_y f_2 of the oracle (2D) or f_1 (1D)."""
    if phys.dim == 1:
        return phys.flux(u, 0)
    return n[0] * phys.flux(u, 0) + n[1] * phys.flux(u, 1)


def _mach3_states():
    """Gas at rest (rho, u, p) = (1, 0, 1) and the state behind a right-moving Mach 3 shock, from
    the normal-shock relations (density, pressure ratio; mass conservation for the velocity)."""
    M2 = 9.0
    c0 = math.sqrt(G)
    s = 3.0 * c0
    rho1 = (G + 1) * M2 / ((G - 1) * M2 + 2)
    p1 = (2 * G * M2 - (G - 1)) / (G + 1)
    u1 = s * (1.0 - 1.0 / rho1)
    cons = lambda r, u, p: torch.tensor([r, r * u, p / (G - 1) + 0.5 * r * u * u], dtype=torch.float64)
    return cons(rho1, u1, p1), cons(1.0, 0.0, 1.0), s


def _dmr_states():
    """The double Mach reflection's post-shock (8, 8.25 cos 30, -8.25 sin 30, 116.5) and pre-shock
    (1.4, 0, 0, 1) states (rho, u, v, p); the shock's normal is (cos 30, -sin 30), speed 10."""
    def cons(r, u, v, p):
        return torch.tensor([r, r * u, r * v, p / (G - 1) + 0.5 * r * (u * u + v * v)], dtype=torch.float64)
    c30, s30 = math.cos(math.pi / 6), math.sin(math.pi / 6)
    return cons(8.0, 8.25 * c30, -8.25 * s30, 116.5), cons(1.4, 0.0, 0.0, 1.0), (c30, -s30), 10.0


def _rh_residual(phys, post, pre, n, s):
    lhs = _flux_n(phys, post, n) - s * post
    rhs = _flux_n(phys, pre, n) - s * pre
    return float(torch.max(torch.abs(lhs - rhs)) / torch.max(torch.abs(lhs)))


def _random_states(dim, seed, count=16):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.3, 3.0, count)
    vel = rng.uniform(-2.0, 2.0, (dim, count))
    p = rng.uniform(0.2, 5.0, count)
    E = p / (G - 1) + 0.5 * rho * np.sum(vel * vel, axis=0)
    u = np.vstack([rho, rho * vel, E])
    return torch.tensor(u, dtype=torch.float64), rho, vel, p


def _jacobian_eigs(phys, u, d):
    J = torch.autograd.functional.jacobian(lambda x: phys.flux(x, d), u)
    return np.sort(np.linalg.eigvals(J.numpy()).real)


def _checks(phys1, phys2):
    """Largest violation of each law (relative), for the 1D and the 2D flux."""
    out = {}
    post, pre, s = _mach3_states()
    out["rh_mach3"] = _rh_residual(phys1, post, pre, None, s)
    post, pre, n, s = _dmr_states()
    out["rh_dmr"] = _rh_residual(phys2, post, pre, n, s)
    worst = 0.0
    for phys, dim in ((phys1, 1), (phys2, 2)):
        U, rho, vel, p = _random_states(dim, 5 + dim)
        for k in range(U.shape[1]):
            c = math.sqrt(G * p[k] / rho[k])
            for d in range(dim):
                un = vel[d, k]
                want = np.sort([un - c, un + c] + [un] * (dim))
                got = _jacobian_eigs(phys, U[:, k].clone(), d)
                worst = max(worst, float(np.max(np.abs(got - want))) / (abs(un) + c))
    out["eigs"] = worst
    U, _, _, _ = _random_states(2, 11)
    # rotate by +90 degrees: (u, v) -> (-v, u); the y-flux of the state is the x-flux of the
    # state rotated by -90 degrees, rotated back
    Ur = torch.stack([U[0], U[2], -U[1], U[3]])          # rotated by -90 degrees
    fx = phys2.flux(Ur, 0)
    back = torch.stack([fx[0], -fx[2], fx[1], fx[3]])    # rotate the vector components back
    fy = phys2.flux(U, 1)
    out["rotation"] = float(torch.max(torch.abs(back - fy)) / torch.max(torch.abs(fy)))
    return out


def test_oracle_euler_flux_obeys_the_physics():
    r = _checks(Euler(1, G), Euler(2, G))
    assert r["rh_mach3"] < 1e-14, r
    assert r["rh_dmr"] < 1e-14, r
    assert r["eigs"] < 1e-12, r
    assert r["rotation"] < 1e-15, r


class _NoPressureEnergy(Euler):
    def flux(self, u, d):
        f = super().flux(u, d)
        p = self.pressure(u)
        return torch.cat([f[:-1], (f[-1] - p * u[1 + d] / u[0])[None]])


class _NoPressureMomentum(Euler):
    def flux(self, u, d):
        f = super().flux(u, d).clone()
        f[1 + d] = f[1 + d] - self.pressure(u)
        return f


class _WrongVelocity(Euler):
    def flux(self, u, d):
        if self.dim == 1:
            return super().flux(u, d)
        return super().flux(u, 1 - d) if d == 1 else super().flux(u, d)


class _WrongGammaFactor(Euler):
    def pressure(self, u):
        return super().pressure(u) * self.gamma / (self.gamma - 1.0) * 0.4


@pytest.mark.parametrize("bad", [_NoPressureEnergy, _NoPressureMomentum, _WrongVelocity, _WrongGammaFactor])
def test_planted_flux_mistakes_are_caught(bad):
    r = _checks(bad(1, G), bad(2, G))
    assert (r["rh_mach3"] > 1e-6 or r["rh_dmr"] > 1e-6 or r["eigs"] > 1e-6 or r["rotation"] > 1e-6), r
