"""Physical fluxes, wave speeds and the quadrature rule used by the oracle.

Test infrastructure: part of the FP64 CPU oracle (see ``oracle/__init__.py``).

* Scalar laws: linear advection f = a u (Sec. 3, eq. 1dlinear), Burgers f = u^2/2
  (Example 4.1).
* Euler equations with ideal-gas law p = (gamma-1)(E - |m|^2/(2 rho)), gamma = 1.4
  unless stated (Sec. 4).  The spectral radius of the flux Jacobian in direction
  n is |u_n| + c with c = sqrt(gamma p / rho) (the Rusanov wave speed of Sec. 2.3).
* Four-point Gauss-Legendre rule in each coordinate (Remark after Algorithm 1),
  written out in closed form on [-1/2, 1/2] with weights summing to one.
* Lax-Friedrichs (Rusanov) flux 1/2 (f(u-) + f(u+)) - 1/2 alpha_d (u+ - u-) with one
  wave speed per direction d: alpha_d = max over the mesh of the spectral radius
  at the cell averages of the state being differentiated (Remark after
  Algorithm 1; the time step of Sec. 4 uses the same "maximum Rusanov wave-speed
  estimates over the mesh").  This global reading reproduces the printed smooth
  Burgers errors of Table 1dBur; a wave speed taken locally at each interface does
  not.

Admissibility: wave speeds are only ever taken at cell averages, so the scheme is
well defined as long as every cell average used has rho > 0 and p > 0; a
violation raises NonPhysicalState.  Point values are not required to be
admissible (their fluxes are plain rational functions).
"""
import math

import torch


class NonPhysicalState(RuntimeError):
    """Raised when a density or pressure is <= 0 (or not finite) at an evaluated point."""


def gauss4():
    """Nodes and weights of the 4-point Gauss-Legendre rule on [-1/2, 1/2]."""
    r = 2.0 / 7.0 * math.sqrt(6.0 / 5.0)
    inner, outer = 0.5 * math.sqrt(3.0 / 7.0 - r), 0.5 * math.sqrt(3.0 / 7.0 + r)
    w_in, w_out = (18.0 + math.sqrt(30.0)) / 72.0, (18.0 - math.sqrt(30.0)) / 72.0
    nodes = [-outer, -inner, inner, outer]
    weights = [w_out, w_in, w_in, w_out]
    return nodes, weights


class Physics:
    """Interface: ncomp, flux(u, d), speed(u, d), check(u).  u has shape [ncomp, ...]."""
    ncomp = 1

    def check(self, u):
        pass


class Advection(Physics):
    def __init__(self, a=(1.0, 0.0)):
        self.a = tuple(float(v) for v in a)
        self.ncomp = 1

    def flux(self, u, d):
        return self.a[d] * u

    def speed(self, u, d):
        return torch.full_like(u[0], abs(self.a[d]))


class Burgers(Physics):
    """f_1 = f_2 = u^2/2."""
    ncomp = 1

    def flux(self, u, d):
        return 0.5 * u * u

    def speed(self, u, d):
        return torch.abs(u[0])


class Euler(Physics):
    """Compressible Euler; dim 1: (rho, m, E); dim 2: (rho, m, n, E)."""

    def __init__(self, dim, gamma=1.4):
        self.dim = dim
        self.gamma = float(gamma)
        self.ncomp = dim + 2

    def pressure(self, u):
        g = self.gamma
        if self.dim == 1:
            rho, m, E = u[0], u[1], u[2]
            return (g - 1.0) * (E - 0.5 * (m * m) / rho)
        rho, m, n, E = u[0], u[1], u[2], u[3]
        return (g - 1.0) * (E - 0.5 * (m * m + n * n) / rho)

    def check(self, u):
        rho = u[0]
        p = self.pressure(u)
        bad = ~(rho > 0) | ~(p > 0)
        if bool(bad.any()):
            raise NonPhysicalState("non-positive density or pressure in a cell average")

    def flux(self, u, d):
        p = self.pressure(u)
        rho, E = u[0], u[-1]
        vel = u[1 + d] / rho
        out = [u[1 + d]]
        for c in range(1, self.dim + 1):
            term = u[c] * vel
            if c == 1 + d:
                term = term + p
            out.append(term)
        out.append((E + p) * vel)
        return torch.stack(out)

    def speed(self, u, d):
        self.check(u)
        p = self.pressure(u)
        rho = u[0]
        return torch.abs(u[1 + d] / rho) + torch.sqrt(self.gamma * p / rho)

    def eigen(self, u, d=0):
        """Left and right eigenvectors of the flux Jacobian in direction d at the states u.

        Textbook forms (the paper uses them for the local characteristic-variable
        FAM5 variant it times in Sec. 4.3 without printing them).  With c the sound
        speed, H = (E + p)/rho the enthalpy, q^2 = |velocity|^2, b1 = (gamma - 1)/c^2
        and b2 = b1 q^2 / 2, the eigenvalues are ordered (u_n - c, u_n, u_n + c) and,
        in 2D, the shear wave u_n last.  Returns (L, R), each [C, C, ...], with
        L = R^{-1} and the columns of R the right eigenvectors.
        """
        g = self.gamma
        C = self.ncomp
        rho = u[0]
        vel = [u[1 + j] / rho for j in range(self.dim)]
        p = self.pressure(u)
        c = torch.sqrt(g * p / rho)
        H = (u[-1] + p) / rho
        q2 = sum(v * v for v in vel)
        b1 = (g - 1.0) / (c * c)
        b2 = 0.5 * b1 * q2
        un = vel[d]
        zero, one = torch.zeros_like(rho), torch.ones_like(rho)
        R = [[zero] * C for _ in range(C)]
        L = [[zero] * C for _ in range(C)]
        # right eigenvectors (columns): acoustic -, entropy, acoustic +
        for col, s in ((0, -1.0), (1, 0.0), (2, 1.0)):
            R[0][col] = one
            for j in range(self.dim):
                R[1 + j][col] = vel[j] + (s * c if j == d else zero)
            R[C - 1][col] = H + s * un * c if s != 0.0 else 0.5 * q2
        # left eigenvectors (rows)
        for row, s in ((0, 1.0), (2, -1.0)):
            L[row][0] = 0.5 * (b2 + s * un / c)
            for j in range(self.dim):
                L[row][1 + j] = -0.5 * (b1 * vel[j] + (s / c if j == d else zero))
            L[row][C - 1] = 0.5 * b1
        L[1][0] = 1.0 - b2
        for j in range(self.dim):
            L[1][1 + j] = b1 * vel[j]
        L[1][C - 1] = -b1
        if self.dim == 2:
            t = 1 - d                      # tangential direction: shear wave
            R[1 + t][3] = one
            R[3][3] = vel[t]
            L[3][0] = -vel[t]
            L[3][1 + t] = one
        return (torch.stack([torch.stack(r) for r in L]), torch.stack([torch.stack(r) for r in R]))


def rusanov(phys, ul, ur, d, alpha):
    """Lax-Friedrichs (Rusanov) flux 1/2 (f(ul) + f(ur)) - 1/2 alpha (ur - ul)."""
    fl, fr = phys.flux(ul, d), phys.flux(ur, d)
    return 0.5 * (fl + fr) - 0.5 * alpha * (ur - ul)


def max_speed(phys, avg, d):
    """alpha_d = max over the given cell averages of the spectral radius in direction d."""
    return torch.max(phys.speed(avg, d))


def make_physics(system, dim, gamma=1.4, a=(1.0, 0.0)):
    if system == "advection":
        return Advection(a)
    if system == "burgers":
        return Burgers()
    if system == "euler":
        return Euler(dim, gamma)
    raise ValueError(f"unknown system {system!r}")
