"""Pins of the oracle's double Mach reflection boundary data (Sec. 4 example) against
the physics they describe, independently of how the oracle builds its ghost cells.

* The two constant states are joined by a shock of normal speed 10 (Mach 10 into gas at
  rest with unit sound speed): the Rankine-Hugoniot conditions F_n(U_post) - s U_post =
  F_n(U_pre) - s U_pre hold with n = (cos 30deg, -sin 30deg), s = 10, and the post-shock
  velocity is along n.
* The top boundary switches from the post- to the pre-shock state where that shock,
  through (1/6, 0) at t = 0 and moving with speed 10 along n, meets the upper edge
  (located from the geometry n . (x - (1/6, 0)) = s t, not from the oracle's formula).
* Below the wall (x > 1/6) the ghost cells hold the moments of the field reflected at
  y = 0 (rho, rho u, E even in y; rho v odd), computed by quadrature of the reflected
  field itself.
"""
import math

import numpy as np
import torch

import fam_inputs as fi
import oracle.scheme as S

N30 = (math.cos(math.pi / 6), -math.sin(math.pi / 6))


def _flux_n(q, n, gamma=1.4):
    rho, mx, my, E = q
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    un = u * n[0] + v * n[1]
    return np.array([rho * un, mx * un + p * n[0], my * un + p * n[1], (E + p) * un])


def test_dmr_states_satisfy_rankine_hugoniot():
    post, pre = (np.array(q) for q in S.dmr_states(1.4))
    c_pre = math.sqrt(1.4 * (0.4 * pre[3]) / pre[0])   # sqrt(gamma p / rho), p = (gamma - 1) E at rest
    assert abs(c_pre - 1.0) < 1e-15
    s = 10.0 * c_pre
    lhs = _flux_n(post, N30) - s * post
    rhs = _flux_n(pre, N30) - s * pre
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
    # the post-shock velocity is normal to the shock
    u, v = post[1] / post[0], post[2] / post[0]
    assert abs(u * N30[1] - v * N30[0]) < 1e-14


def test_top_boundary_follows_the_moving_shock():
    nx, ny = 300, 100
    cfg = S.Config(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", dmr=True)
    U = torch.tensor(fi.double_mach(nx, ny))
    post, pre = S.dmr_states(1.4)
    xc = (np.arange(nx) + 0.5) * cfg.dx
    for t in (0.0, 0.013, 0.05, 0.14, 0.2):   # by t = 0.2 the shock has left through the top edge
        P = S.pad(U, cfg, t=t)
        for row in (-1, -2):
            top = P[0, 0, row, 2:-2].numpy()
            is_post = top == post[0]
            assert np.all(is_post | (top == pre[0]))
            # post-shock on the left of the crossing, pre-shock on its right
            k = int(np.argmin(is_post)) if not is_post.all() else nx
            assert np.all(is_post[:k]) and not np.any(is_post[k:])
            y_top = cfg.y1
            x_cross = 1.0 / 6.0 + (10.0 * t - N30[1] * y_top) / N30[0]   # n . (x - (1/6, 0)) = 10 t
            lo = xc[k - 1] if k > 0 else -np.inf
            hi = xc[k] if k < nx else np.inf
            assert lo < x_cross <= hi + 1e-12


def test_reflecting_wall_ghosts_are_moments_of_the_mirrored_field():
    nx, ny = 60, 20
    cfg = S.Config(dim=2, nx=nx, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", dmr=True)

    def field(X, Y):
        rho = 1.5 + 0.3 * np.sin(2.0 * X + 1.0) * np.cos(3.0 * Y + 0.4)
        m = 0.7 + 0.2 * np.cos(X - 2.0 * Y)
        n = 0.4 * np.sin(1.5 * X + 2.5 * Y + 0.3)
        E = 4.0 + 0.5 * np.cos(0.7 * X * Y + Y)
        return np.stack([rho, m, n, E])

    def mirrored(X, Y):
        f = field(X, -Y)
        f[2] = -f[2]
        return f

    U = fi.moments_2d(field, 0.0, 3.0, 0.0, 1.0, nx, ny)
    ghost = fi.moments_2d(mirrored, 0.0, 3.0, -2.0 * cfg.dy, 0.0, nx, 2)     # rows r = -2, -1
    P = S.pad(torch.tensor(U), cfg, t=0.0).numpy()
    xc = (np.arange(nx) + 0.5) * cfg.dx
    wall = xc > 1.0 / 6.0
    got = P[:, :, 0:2, 2:-2][..., wall]
    ref = ghost[..., wall]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # left of x = 1/6 the bottom ghosts hold the post-shock state with zero first moments
    post = S.dmr_states(1.4)[0]
    for c in range(4):
        assert np.all(P[c, 0, 0:2, 2:-2][:, ~wall] == post[c])
        assert np.all(P[c, 1:, 0:2, 2:-2][..., ~wall] == 0.0)


def test_shu_osher_left_state_is_the_mach3_post_shock_state():
    """The Shu-Osher-type workload's left state (printed to 6-7 digits) and the gas at rest
    ahead of it, (1, 0, 1), satisfy the 1D Rankine-Hugoniot conditions of a shock moving
    right at Mach 3 (speed 3 sqrt(1.4)), to the printed precision."""
    rl, ul, pl = fi.SHU_OSHER_LEFT
    g = 1.4
    s = 3.0 * math.sqrt(g * 1.0 / 1.0)

    def F(rho, u, p):
        E = p / (g - 1.0) + 0.5 * rho * u * u
        return np.array([rho * u, rho * u * u + p, (E + p) * u]) - s * np.array([rho, rho * u, E])

    left, right = F(rl, ul, pl), F(1.0, 0.0, 1.0)
    assert np.max(np.abs(left - right) / np.abs(right)) < 5e-6   # p is printed as 10.33333
    # and the printed values are those of the exact Mach 3 jump to their last digit
    M2 = 9.0
    assert abs(rl - (g + 1) * M2 / ((g - 1) * M2 + 2)) < 1e-6
    assert abs(pl - (2 * g * M2 - (g - 1)) / (g + 1)) < 1e-5
    assert abs(ul - s * (1.0 - 1.0 / ((g + 1) * M2 / ((g - 1) * M2 + 2)))) < 1e-6
