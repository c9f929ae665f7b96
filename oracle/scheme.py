"""The FAM time step written out as plain FP64 array operations over all cells.

Test infrastructure: part of the FP64 CPU oracle (see ``oracle/__init__.py``).

State layout: a tensor U[c, r, ...] with component c and moment r (r = 0 cell
average, r = 1 scaled x-moment, r = 2 scaled y-moment), followed by the cell
indices ([nx] in 1D, [ny, nx] in 2D).

One step (Algorithm 1 for 1D, system (12) for 2D):

1. time step from the cell averages: dt = C dx / alpha_x (1D) or
   dt = C / (alpha_x/dx + alpha_y/dy) (2D), alpha = max wave speed over the mesh
   (the "discontinuous problems" rule of Sec. 4);
2. three SSP-RK3 stages in Shu-Osher form (eqs. 3 and 12), each evaluating the
   semi-discrete operator R of eq. (1dSemi) / eq. (11): componentwise compact
   reconstruction, Lax-Friedrichs (Rusanov) flux at the 4 Gauss points of each
   face with alpha_d = max over the mesh of the spectral radius at the stage
   state's cell averages, 4x4 Gauss volume quadrature of the first-moment volume
   term;
3. one OE pass (Prop. 2.1, eq. 1dOE_system; eq. 2dOE_sol, eq. 2dOE_system) with
   the Type I or Type II damping coefficients of Tables sigma1d / sigma2d.

Boundary treatment: two ghost layers, periodic wrap or transmissive copy of every
moment of the nearest interior cell (Remark after Algorithm 1).
"""
from dataclasses import dataclass, field

import math

import torch

from . import exact
from .physics import gauss4, make_physics, max_speed, rusanov

DT = torch.float64

# default OE constants gamma_k: Sec. 2.1 (1D) and Sec. 2.2 (2D)
GAMMA_K_1D = {3: 25.0, 4: 25.0, 5: 12.5, 6: 12.5}
GAMMA_K_2D = {3: 25.0, 4: 25.0, 5: 15.0, 6: 15.0}


@dataclass
class Config:
    dim: int
    nx: int
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    k: int = 5
    system: str = "euler"          # advection | burgers | euler
    gamma: float = 1.4
    a: tuple = (1.0, 0.0)          # advection velocity
    bc_x: str = "periodic"         # periodic | transmissive
    bc_y: str = "periodic"
    oe: str = "type2"              # off | type1 | type2
    oe_gamma_k: float = 0.0        # <= 0: the paper's default for (dim, k)
    cfl: float = 0.2
    k6_jump_from_table: bool = False
    pp: bool = False               # positivity limiter on the stage reconstruction (Euler)
    dt_rule: int = 0               # 0: C dx / alpha; 1: C dx^{k/3} / alpha (smooth tests, Sec. 4)
    dmr: bool = False              # double Mach reflection boundaries (Sec. 4 example)
    char_vars: bool = False        # stage reconstruction in local characteristic variables (Euler)
    phys: object = field(default=None, repr=False)

    def __post_init__(self):
        if self.dim == 1:
            self.ny = 1
        self.phys = make_physics(self.system, self.dim, self.gamma, self.a)
        if self.char_vars and self.system != "euler":
            raise ValueError("characteristic variables need the Euler equations")

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def ncomp(self):
        return self.phys.ncomp

    @property
    def gamma_k(self):
        if self.oe_gamma_k > 0:
            return self.oe_gamma_k
        return (GAMMA_K_1D if self.dim == 1 else GAMMA_K_2D)[self.k]

    def state_shape(self):
        if self.dim == 1:
            return (self.ncomp, 2, self.nx)
        return (self.ncomp, 3, self.ny, self.nx)


# ----------------------------------------------------------------------------
# ghost cells
# ----------------------------------------------------------------------------
def _ghost_index(n, g, bc):
    idx = torch.arange(-g, n + g)
    if bc == "periodic":
        return idx % n
    if bc == "transmissive":
        return idx.clamp(0, n - 1)
    raise ValueError(f"unknown boundary condition {bc!r}")


def pad(U, cfg, g=2, t=0.0):
    """Return U with g ghost layers on every side (layout preserved); t is the time of
    time-dependent boundary data (the double Mach reflection's upper boundary)."""
    if cfg.dmr:
        return _pad_dmr(U, cfg, g, t)
    ix = _ghost_index(cfg.nx, g, cfg.bc_x)
    if cfg.dim == 1:
        return U[..., ix]
    iy = _ghost_index(cfg.ny, g, cfg.bc_y)
    return U[..., iy, :][..., ix]


def dmr_states(gamma):
    """Conservative states behind and ahead of the incident Mach 10 shock of the double
    Mach reflection example (Sec. 4): (rho, u, v, p) = (8, 8.25 cos 30deg, -8.25 sin 30deg,
    116.5) and (1.4, 0, 0, 1)."""
    out = []
    for rho, u, v, p in ((8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5),
                         (1.4, 0.0, 0.0, 1.0)):
        out.append([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
    return out


def _pad_dmr(U, cfg, g, t):
    """Ghost cells of the double Mach reflection example, cell by cell:
    * above the mesh, the exact moving shock: post-shock state where the cell centre
      lies left of x = 1/6 + (y1 + 20 t) / sqrt(3), pre-shock state beyond;
    * below the mesh, the post-shock state where the cell centre has x < 1/6, else a
      reflecting wall: the mirror image of the interior row, with the average and
      x-moment of rho v and the y-moments of rho, rho u, E negated;
    * left of the mesh, the post-shock state; right of it, a copy of the last column.
    Constant states have zero first moments."""
    post, pre = dmr_states(cfg.gamma)
    C, M, ny, nx = U.shape
    out = torch.empty((C, M, ny + 2 * g, nx + 2 * g), dtype=U.dtype)
    xs = 1.0 / 6.0 + (cfg.y1 + 20.0 * t) / math.sqrt(3.0)
    const = lambda q: torch.tensor([[q[c], 0.0, 0.0][m] for c in range(C) for m in range(M)],
                                   dtype=U.dtype).reshape(C, M)
    Qpost, Qpre = const(post), const(pre)
    for jj in range(ny + 2 * g):
        r = jj - g
        for ii in range(nx + 2 * g):
            ci = ii - g
            xc = cfg.x0 + (ci + 0.5) * cfg.dx
            if r >= ny:
                out[:, :, jj, ii] = Qpost if xc < xs else Qpre
                continue
            if (r < 0 and xc < 1.0 / 6.0) or (r >= 0 and ci < 0):
                out[:, :, jj, ii] = Qpost
                continue
            gi = min(ci, nx - 1)
            if r < 0:
                v = U[:, :, -1 - r, gi].clone()
                v[2, 0] = -v[2, 0]
                v[2, 1] = -v[2, 1]
                v[0, 2], v[1, 2], v[3, 2] = -v[0, 2], -v[1, 2], -v[3, 2]
                out[:, :, jj, ii] = v
            else:
                out[:, :, jj, ii] = U[:, :, r, gi]
    return out


# ----------------------------------------------------------------------------
# reconstruction (Sec. 2.4): exact operators rounded once to FP64
# ----------------------------------------------------------------------------
_OPS = {}


def recon_matrix(dim, k, full_aux=False):
    key = (dim, k, full_aux)
    if key not in _OPS:
        if full_aux:
            monos, R = exact.space_2d(k), exact.aux_operator(dim, k)
        else:
            monos, R = exact.recon_operator(dim, k)
        _OPS[key] = (monos, torch.tensor([[float(v) for v in row] for row in R], dtype=DT))
    return _OPS[key]


def eval_matrix(monos, points):
    """E[q, m] = value of monomial m at point q."""
    rows = []
    for pt in points:
        row = []
        for m in monos:
            v = 1.0
            for e, x in zip(m, pt):
                v *= x ** e
            row.append(v)
        rows.append(row)
    return torch.tensor(rows, dtype=DT)


def stencil_1d(Upad, k):
    """Stencil inputs (constraint order of eq. 5 / eq. 6) for cells 1..n+2 of the 2-ghost pad.

    Upad: [C, 2, n+4]; returns [C, ninputs, n+2] for the cells with one-ring
    (indices -1..n in interior numbering).
    """
    n2 = Upad.shape[-1] - 2
    cols = []
    for a, kind in exact.constraints_1d(k):
        cols.append(Upad[:, kind, 1 + a: 1 + a + n2])
    return torch.stack(cols, dim=1)


def stencil_2d(Upad, k):
    """Stencil inputs (constraint order of systems Qxy_quartic / Qxy_quintic).

    Upad: [C, 3, ny+4, nx+4]; returns [C, ninputs, ny+2, nx+2] for the interior
    cells and their one-ring.
    """
    H, W = Upad.shape[-2] - 2, Upad.shape[-1] - 2
    cols = []
    for l, kind in exact.constraints_2d(k):
        a, b = exact.PATCH_OFFSETS[l]
        cols.append(Upad[:, kind, 1 + b: 1 + b + H, 1 + a: 1 + a + W])
    return torch.stack(cols, dim=1)


def reconstruct(Upad, cfg, full_aux=False):
    """Monomial coefficients of p_k (or of the auxiliary Q) on interior cells + one ring."""
    monos, R = recon_matrix(cfg.dim, cfg.k, full_aux)
    S = stencil_1d(Upad, cfg.k) if cfg.dim == 1 else stencil_2d(Upad, cfg.k)
    coef = torch.einsum("pi,ci...->cp...", R, S)
    return monos, coef


def reconstruct_stage(Upad, cfg):
    """The RK-stage reconstruction: componentwise in conservative variables, or with
    cfg.char_vars in the local characteristic variables of each cell.

    The characteristic variant (the FAM5 alternative timed in Sec. 4.3, Table
    runtime-main Panel B): every cell maps its whole stencil of moments to the
    characteristic variables of its own cell average with the left eigenvectors
    of the x-direction flux Jacobian there, reconstructs each characteristic
    field with the same linear operator, and maps the polynomial's coefficients
    back with the right eigenvectors.  Sec. 2.3 notes that a linear reconstruction
    commutes with a fixed change of variables, so both give the same polynomial
    up to rounding; the variant only changes the cost.
    """
    if not cfg.char_vars:
        return reconstruct(Upad, cfg)
    monos, Rm = recon_matrix(cfg.dim, cfg.k)
    S = stencil_1d(Upad, cfg.k) if cfg.dim == 1 else stencil_2d(Upad, cfg.k)
    avg = Upad[:, 0, 1:-1] if cfg.dim == 1 else Upad[:, 0, 1:-1, 1:-1]   # the stencils' own cells
    L, R = cfg.phys.eigen(avg, 0)
    W = torch.einsum("ab...,bi...->ai...", L, S)           # characteristic stencil values
    coef_w = torch.einsum("pi,ai...->ap...", Rm, W)        # reconstruct each field
    return monos, torch.einsum("ca...,ap...->cp...", R, coef_w)


def point_values(monos, coef, points):
    E = eval_matrix(monos, points)
    return torch.einsum("qp,cp...->cq...", E, coef)


# ----------------------------------------------------------------------------
# optional positivity safeguard on the stage reconstruction
# ----------------------------------------------------------------------------
def pp_theta(vals, avg, phys):
    """Scaling factor theta in [0, 1] of the positivity limiter for every cell.

    The paper applies an auxiliary BP/PP limiter in some tests but does not give
    its algorithm; this is the classical scaling limiter: the reconstruction p is
    replaced by avg + theta (p - avg), with theta the largest value keeping density
    and pressure >= eps = min(1e-13, rho_avg, p(avg)) at every point where a flux
    is evaluated (vals: [C, Q, ...]).  Density is limited first (theta_1), then
    pressure along the segment from avg to the density-limited point values.
    """
    g = phys.gamma
    rho_a = avg[0]
    p_a = phys.pressure(avg)
    if bool((~(rho_a > 0) | ~(p_a > 0)).any()):
        from .physics import NonPhysicalState
        raise NonPhysicalState("non-positive cell-average density or pressure")
    eps = torch.clamp(torch.minimum(rho_a, p_a), max=1e-13)
    rho_min = torch.min(vals[0], dim=0).values
    lim1 = rho_min < eps
    den1 = torch.where(lim1, rho_a - rho_min, torch.ones_like(rho_a))
    theta1 = torch.where(lim1, (rho_a - eps) / den1, torch.ones_like(rho_a))
    w = vals.clone()
    w[0] = rho_a.unsqueeze(0) + theta1.unsqueeze(0) * (vals[0] - rho_a.unsqueeze(0))
    # pressure: t_q solves p(avg + t (w_q - avg)) = eps on (0, 1] where p(w_q) < eps
    d = w - avg.unsqueeze(1)
    A = avg.unsqueeze(1)
    rho0, E0, rhod, Ed = A[0], A[-1], d[0], d[-1]
    mom0, momd = A[1:-1], d[1:-1]
    kk = 2.0 / (g - 1.0)
    qa = 2.0 * rhod * Ed - (momd * momd).sum(dim=0)
    qb = 2.0 * (rho0 * Ed + rhod * E0) - 2.0 * (mom0 * momd).sum(dim=0) - kk * eps.unsqueeze(0) * rhod
    qc = 2.0 * rho0 * E0 - (mom0 * mom0).sum(dim=0) - kk * eps.unsqueeze(0) * rho0
    p_w = phys.pressure(w)
    need = p_w < eps.unsqueeze(0)
    t = _smallest_root_in_unit(qa, qb, qc, need)
    theta2 = torch.min(t, dim=0).values
    return theta1, theta2


def _smallest_root_in_unit(a, b, c, need):
    """Smallest root in (0, 1] of a t^2 + b t + c (c > 0, value <= 0 at t = 1) where need, else 1."""
    one = torch.ones_like(c)
    disc = torch.clamp(b * b - 4.0 * a * c, min=0.0)
    sq = torch.sqrt(disc)
    sgn = torch.where(b >= 0, one, -one)
    q = -0.5 * (b + sgn * sq)
    q_safe = torch.where(q == 0, one, q)
    a_safe = torch.where(a == 0, one, a)
    r1 = torch.where(a == 0, torch.full_like(c, 2.0), q / a_safe)
    r2 = c / q_safe
    big = torch.full_like(c, 2.0)
    r1 = torch.where((r1 > 0) & (r1 <= 1), r1, big)
    r2 = torch.where((r2 > 0) & (r2 <= 1), r2, big)
    r = torch.minimum(r1, r2)
    r = torch.where(r > 1, one, r)
    return torch.where(need, r, one)


def pp_apply(vals, avg, theta1, theta2):
    """Point values of the limited reconstruction avg + theta2 (w - avg); cells with
    theta1 = theta2 = 1 keep their point values unchanged."""
    A = avg.unsqueeze(1)
    w = vals.clone()
    w[0] = A[0] + theta1.unsqueeze(0) * (vals[0] - A[0])
    lim = A + theta2.unsqueeze(0) * (w - A)
    active = ((theta1 < 1) | (theta2 < 1)).unsqueeze(0).unsqueeze(0)
    return torch.where(active, lim, vals)


# ----------------------------------------------------------------------------
# semi-discrete operator R(U)
# ----------------------------------------------------------------------------
def residual_1d(U, cfg, t=0.0):
    """R(U) of eq. (1dSemi) for every cell: returns [C, 2, n]."""
    phys = cfg.phys
    nodes, weights = gauss4()
    Upad = pad(U, cfg)
    monos, coef = reconstruct_stage(Upad, cfg)            # cells -1..n
    pts = [(0.5,), (-0.5,)] + [(x,) for x in nodes]
    vals = point_values(monos, coef, pts)                  # [C, 6, n+2]
    if cfg.pp:
        avg = Upad[:, 0, 1:-1]
        th1, th2 = pp_theta(vals, avg, phys)
        vals = pp_apply(vals, avg, th1, th2)
    right, left = vals[:, 0], vals[:, 1]
    alpha = max_speed(phys, U[:, 0], 0)
    # interface i+1/2 for i = -1..n-1: left state = right trace of cell i
    fhat = rusanov(phys, right[:, :-1], left[:, 1:], 0, alpha)  # [C, n+1]
    vol = vals[:, 2:, 1:-1]                                # [C, 4, n]
    V = sum(weights[g] * phys.flux(vol[:, g], 0) for g in range(4))
    dx = cfg.dx
    R0 = -(fhat[:, 1:] - fhat[:, :-1]) / dx
    R1 = (V - 0.5 * (fhat[:, 1:] + fhat[:, :-1])) / dx
    return torch.stack([R0, R1], dim=1)


def points_2d():
    """The 32 flux-evaluation points of a cell, in this order: right face (1/2, eta_g),
    left face (-1/2, eta_g), top face (xi_g, 1/2), bottom face (xi_g, -1/2), then the
    4x4 volume points (xi_a, eta_b) with index 16 + 4 b + a."""
    nodes, _ = gauss4()
    pts = [(0.5, e) for e in nodes] + [(-0.5, e) for e in nodes]
    pts += [(e, 0.5) for e in nodes] + [(e, -0.5) for e in nodes]
    pts += [(nodes[a], nodes[b]) for b in range(4) for a in range(4)]
    return pts


def residual_2d(U, cfg, t=0.0):
    """R(U) of eq. (11) on the Cartesian mesh: returns [C, 3, ny, nx]."""
    phys = cfg.phys
    nodes, weights = gauss4()
    Upad = pad(U, cfg, t=t)
    monos, coef = reconstruct_stage(Upad, cfg)             # [C, P, ny+2, nx+2]
    vals = point_values(monos, coef, points_2d())          # [C, 32, ny+2, nx+2]
    if cfg.pp:
        avg = Upad[:, 0, 1:-1, 1:-1]
        th1, th2 = pp_theta(vals, avg, phys)
        vals = pp_apply(vals, avg, th1, th2)
    ax, ay = max_speed(phys, U[:, 0], 0), max_speed(phys, U[:, 0], 1)
    # x-interfaces (i+1/2, j) for i = -1..nx-1, interior rows
    right = vals[:, 0:4, 1:-1, :]
    left = vals[:, 4:8, 1:-1, :]
    Fhat = torch.stack([rusanov(phys, right[:, g, :, :-1], left[:, g, :, 1:], 0, ax)
                        for g in range(4)], dim=1)                 # [C, 4, ny, nx+1]
    Fbar = sum(weights[g] * Fhat[:, g] for g in range(4))
    Ftil = sum(weights[g] * nodes[g] * Fhat[:, g] for g in range(4))
    # y-interfaces (i, j+1/2) for j = -1..ny-1, interior columns
    top = vals[:, 8:12, :, 1:-1]
    bot = vals[:, 12:16, :, 1:-1]
    Ghat = torch.stack([rusanov(phys, top[:, g, :-1, :], bot[:, g, 1:, :], 1, ay)
                        for g in range(4)], dim=1)                 # [C, 4, ny+1, nx]
    Gbar = sum(weights[g] * Ghat[:, g] for g in range(4))
    Gtil = sum(weights[g] * nodes[g] * Ghat[:, g] for g in range(4))
    # 4x4 volume quadrature of the first-moment volume terms
    vol = vals[:, 16:32, 1:-1, 1:-1]                               # [C, 16, ny, nx]
    V1 = sum(weights[q % 4] * weights[q // 4] * phys.flux(vol[:, q], 0) for q in range(16))
    V2 = sum(weights[q % 4] * weights[q // 4] * phys.flux(vol[:, q], 1) for q in range(16))
    dx, dy = cfg.dx, cfg.dy
    R0 = -(Fbar[..., 1:] - Fbar[..., :-1]) / dx - (Gbar[:, 1:] - Gbar[:, :-1]) / dy
    R1 = V1 / dx - (Fbar[..., 1:] + Fbar[..., :-1]) / (2 * dx) - (Gtil[:, 1:] - Gtil[:, :-1]) / dy
    R2 = V2 / dy - (Gbar[:, 1:] + Gbar[:, :-1]) / (2 * dy) - (Ftil[..., 1:] - Ftil[..., :-1]) / dx
    return torch.stack([R0, R1, R2], dim=1)


def residual(U, cfg, t=0.0):
    return residual_1d(U, cfg) if cfg.dim == 1 else residual_2d(U, cfg, t)


# ----------------------------------------------------------------------------
# time step and SSP-RK3
# ----------------------------------------------------------------------------
def cfl_dt(U, cfg):
    """Time step of Sec. 4 from the cell averages: C dx / alpha for the discontinuous
    problems, or C dx^{k/3} / alpha for the smooth accuracy tests (dt_rule = 1); in 2D
    C / (alpha_x / hx + alpha_y / hy) with hx, hy those lengths."""
    avg = U[:, 0]
    ax = max_speed(cfg.phys, avg, 0)
    e = cfg.k / 3.0 if cfg.dt_rule == 1 else 1.0
    if cfg.dim == 1:
        return float(cfg.cfl * cfg.dx ** e / ax)
    ay = max_speed(cfg.phys, avg, 1)
    return float(cfg.cfl / (ax / cfg.dx ** e + ay / cfg.dy ** e))


STAGE_TIME = (0.0, 1.0, 0.5)   # stage s evaluates R at t_n + STAGE_TIME[s] dt


RK3_C0 = (0.0, 0.75, 1.0 / 3.0)   # weight of U^n in stage s; L = U^s + dt R(U^s) gets 1 - c


def rk3_stage(s, U0, Us, dt, cfg, t=0.0):
    """Stage s (0, 1, 2) of the Shu-Osher form of SSP-RK3 (eq. 12); t = t_n (boundary data).

    The convex combination c U0 + (1 - c) L is evaluated as L + c (U0 - L).  Written
    with the two weights rounded separately, the last stage's 1/3 and 2/3 sum to
    1 - 2^-54 in FP64, which shrinks every value by that factor in every step: on a
    smooth run of 5.7e4 steps a bias of 3e-12 in the density, larger than the printed
    FAM6 error of Table 1dEuler at N = 70 (the bias doubles when dt is halved)."""
    Ls = Us + dt * residual(Us, cfg, t + STAGE_TIME[s] * dt)
    if s == 0:
        return Ls
    return Ls + RK3_C0[s] * (U0 - Ls)


def rk3(U0, dt, cfg, t=0.0):
    U1 = rk3_stage(0, U0, U0, dt, cfg, t)
    U2 = rk3_stage(1, U0, U1, dt, cfg, t)
    return rk3_stage(2, U0, U2, dt, cfg, t)


# ----------------------------------------------------------------------------
# oscillation elimination
# ----------------------------------------------------------------------------
def _sigma(J, avg_patch, cfg, global_stats):
    """Scalar damping coefficients of Table sigma1d / sigma2d for every cell.

    J: jump accumulation(s) [C, ...]; avg_patch: [C, |Lambda|, ...] cell averages over
    Lambda; global_stats: (D_Omega, eps_Omega) per component for Type I.
    """
    if cfg.oe == "type2":
        S = avg_patch.sum(dim=1)
        D = torch.max(torch.abs(avg_patch - S.unsqueeze(1)), dim=1).values
        eps = 1e-14 * torch.clamp(torch.max(torch.abs(avg_patch), dim=1).values, min=1.0)
    else:
        D_om, eps_om = global_stats
        shape = (-1,) + (1,) * (J.dim() - 1)
        D = D_om.reshape(shape).expand_as(J)
        eps = eps_om.reshape(shape).expand_as(J)
    small = D < eps
    D_safe = torch.where(small, torch.ones_like(D), D)
    return torch.where(small, torch.zeros_like(J), cfg.gamma_k * J / D_safe)


def _type1_stats(avg):
    """Global reference quantities of Type I: D_Omega and eps_Omega per component."""
    C = avg.shape[0]
    flat = avg.reshape(C, -1)
    mean = flat.sum(dim=1) / flat.shape[1]
    D = torch.max(torch.abs(flat - mean[:, None]), dim=1).values
    eps = 1e-14 * torch.clamp(torch.max(torch.abs(flat), dim=1).values, min=1.0)
    return D, eps


def _jump_monos_coef(Upad, cfg):
    use_aux = cfg.dim == 2 and cfg.k == 6 and cfg.k6_jump_from_table
    return reconstruct(Upad, cfg, full_aux=use_aux)


def oe_1d(Un, dt, cfg):
    """OE pass of eq. (1dOE_system) (scalar case: eq. 9)."""
    if cfg.oe == "off":
        return Un
    delta = oe_delta_1d(Un, dt, cfg)
    return torch.stack([Un[:, 0], Un[:, 1] * delta], dim=1)


def oe_delta_1d(Un, dt, cfg):
    """Damping factor delta of every cell in the OE pass of eq. (1dOE_system)."""
    phys = cfg.phys
    Upad = pad(Un, cfg)
    monos, coef = _jump_monos_coef(Upad, cfg)               # cells -1..n
    right = point_values(monos, coef, [(0.5,)])[:, 0]
    left = point_values(monos, coef, [(-0.5,)])[:, 0]
    jump = left[:, 1:] - right[:, :-1]                       # interfaces -1/2 .. n-1/2
    J = torch.abs(jump[:, :-1]) + torch.abs(jump[:, 1:])     # [C, n]
    n = cfg.nx
    avgp = Upad[:, 0]                                        # [C, n+4]
    patch = torch.stack([avgp[:, 2 + a: 2 + a + n] for a in (-1, 0, 1)], dim=1)
    stats = _type1_stats(Un[:, 0]) if cfg.oe == "type1" else None
    sig = torch.max(_sigma(J, patch, cfg, stats), dim=0).values
    speeds = torch.stack([phys.speed(patch[:, m], 0) for m in range(3)])
    beta = torch.max(speeds, dim=0).values
    return torch.exp(-beta * dt * sig / cfg.dx)


def oe_2d(Un, dt, cfg, t=0.0):
    """OE pass of eq. (2dOE_system) with the common factor delta_{i,j}; t: time of Un."""
    if cfg.oe == "off":
        return Un
    delta = oe_delta_2d(Un, dt, cfg, t)
    return torch.stack([Un[:, 0], Un[:, 1] * delta, Un[:, 2] * delta], dim=1)


def oe_delta_2d(Un, dt, cfg, t=0.0):
    """Damping factor delta_{i,j} of every cell in the OE pass of eq. (2dOE_system)."""
    phys = cfg.phys
    Upad = pad(Un, cfg, t=t)
    monos, coef = _jump_monos_coef(Upad, cfg)                # [C, P, ny+2, nx+2]
    cx = coef[:, :, 1:-1, :]
    r = point_values(monos, cx, [(0.5, 0.0)])[:, 0]
    l = point_values(monos, cx, [(-0.5, 0.0)])[:, 0]
    jx = l[..., 1:] - r[..., :-1]                             # [C, ny, nx+1]
    Jx = torch.abs(jx[..., :-1]) + torch.abs(jx[..., 1:])
    cy = coef[:, :, :, 1:-1]
    t = point_values(monos, cy, [(0.0, 0.5)])[:, 0]
    b = point_values(monos, cy, [(0.0, -0.5)])[:, 0]
    jy = b[:, 1:] - t[:, :-1]                                 # [C, ny+1, nx]
    Jy = torch.abs(jy[:, :-1]) + torch.abs(jy[:, 1:])
    ny, nx = cfg.ny, cfg.nx
    avgp = Upad[:, 0]
    patch = torch.stack([avgp[:, 2 + bb: 2 + bb + ny, 2 + aa: 2 + aa + nx]
                         for l_ in range(1, 10)
                         for aa, bb in [exact.PATCH_OFFSETS[l_]]], dim=1)  # [C, 9, ny, nx]
    stats = _type1_stats(Un[:, 0]) if cfg.oe == "type1" else None
    sx = torch.max(_sigma(Jx, patch, cfg, stats), dim=0).values
    sy = torch.max(_sigma(Jy, patch, cfg, stats), dim=0).values
    bx = torch.max(torch.stack([phys.speed(patch[:, m], 0) for m in range(9)]), dim=0).values
    by = torch.max(torch.stack([phys.speed(patch[:, m], 1) for m in range(9)]), dim=0).values
    return torch.exp(-bx * dt * sx / cfg.dx - by * dt * sy / cfg.dy)


def oe(Un, dt, cfg, t=0.0):
    return oe_1d(Un, dt, cfg) if cfg.dim == 1 else oe_2d(Un, dt, cfg, t)


def oe_delta(Un, dt, cfg, t=0.0):
    return oe_delta_1d(Un, dt, cfg) if cfg.dim == 1 else oe_delta_2d(Un, dt, cfg, t)


# ----------------------------------------------------------------------------
# driver
# ----------------------------------------------------------------------------
def step(U, cfg, dt=None, t=0.0):
    """One FAM step from time t; dt=None computes the CFL time step from U.
    Returns (U_new, dt)."""
    if dt is None:
        dt = cfl_dt(U, cfg)
    Un = rk3(U, dt, cfg, t)
    return oe(Un, dt, cfg, t + dt), dt


def run(U, cfg, nsteps=None, t_final=None, dt=None):
    """Advance nsteps steps, or until t_final (last step clipped to land on it)."""
    t = 0.0
    steps = 0
    while True:
        if nsteps is not None and steps >= nsteps:
            break
        if t_final is not None and t >= t_final:
            break
        h = dt if dt is not None else cfl_dt(U, cfg)
        if t_final is not None and t + h > t_final:
            h = t_final - t
        U, _ = step(U, cfg, h, t)
        t += h
        steps += 1
    return U, t, steps


def as_tensor(U):
    if isinstance(U, torch.Tensor):
        return U.to(dtype=DT, device="cpu")
    return torch.as_tensor(U, dtype=DT)
