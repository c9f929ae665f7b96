"""Final-time functional and its reference gradient (oracle side).

Test infrastructure: part of the FP64 CPU oracle (see ``oracle/__init__.py``).

J(U_T) = integral over [1/4, 3/4]^2 of rho_h(T)^2, where rho_h is the local P1
moment representation u^(0) + 12 u^(1) xi + 12 u^(2) eta of the evolved state
(Sec. 2.1: int phi^(1)^2 = dx/12).  Over one cell this integral is exactly
dx dy (u0^2 + 12 u1^2 + 12 u2^2).  Cells whose centres lie in the window count.

The reference gradient dJ/dU_0 differentiates the oracle's own FAM steps with
torch's reverse mode (time step held fixed).  Non-smooth points follow torch's
rules for the operations the oracle uses: |x|' = sign(x) with sign(0) = 0,
``torch.where`` and ``torch.max(dim)`` pass the derivative to the selected /
first maximal entry, and the eps-branch of the OE coefficient has derivative 0.
"""
import torch

from .scheme import as_tensor, step


def window_mask(cfg, lo=0.25, hi=0.75):
    xc = cfg.x0 + (torch.arange(cfg.nx, dtype=torch.float64) + 0.5) * cfg.dx
    yc = cfg.y0 + (torch.arange(cfg.ny, dtype=torch.float64) + 0.5) * cfg.dy
    mx = (xc >= lo) & (xc <= hi)
    my = (yc >= lo) & (yc <= hi)
    return (my[:, None] & mx[None, :]).to(torch.float64)


def functional(U, cfg):
    """J = sum over window cells of dx dy (rho0^2 + 12 rho1^2 + 12 rho2^2)."""
    m = window_mask(cfg)
    rho = U[0]
    return cfg.dx * cfg.dy * torch.sum(m * (rho[0] ** 2 + 12.0 * rho[1] ** 2 + 12.0 * rho[2] ** 2))


def run_fixed(U0, cfg, nsteps, dt):
    U = U0
    for _ in range(nsteps):
        U, _ = step(U, cfg, dt)
    return U


def reference_gradient(U0, cfg, nsteps, dt):
    """(J, dJ/dU0) by reverse-mode differentiation of nsteps oracle steps."""
    U = as_tensor(U0).clone().requires_grad_(True)
    J = functional(run_fixed(U, cfg, nsteps, dt), cfg)
    (g,) = torch.autograd.grad(J, U)
    return float(J.detach()), g.detach()


def directional_derivative(U0, cfg, nsteps, dt, direction):
    """Exact directional derivative dJ/dU0 . direction by forward-mode (dual numbers)."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        U = fwAD.make_dual(as_tensor(U0), as_tensor(direction))
        J = functional(run_fixed(U, cfg, nsteps, dt), cfg)
        return float(fwAD.unpack_dual(J).tangent)
