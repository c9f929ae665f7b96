"""The transmissive boundary reading (every moment of the nearest interior cell copied into the
ghost layers, corners by clamping both indices) pinned through the periodic operator, which the
Fourier tests pin: for one evaluation of the residual (eq. 11), transmissive ghosts must act
exactly like real cells holding those copies.  So the residual of a mesh with transmissive
boundaries equals, on the mesh's own cells, the residual of the same mesh extended on every side
by three layers of copies of its edge cells and closed periodically (the wrap-around is then
further away than the stencil and flux reach of every original cell).

Planted mistakes in the oracle's ghost cells (the second cell copied instead of the first, the
ghost moments zeroed, the x and y rules swapped) fail the comparison.
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S

EXT = 3


def _extend_1d(U):
    left = U[..., :1].repeat_interleave(EXT, dim=-1)
    right = U[..., -1:].repeat_interleave(EXT, dim=-1)
    return torch.cat([left, U, right], dim=-1)


def _extend_2d(U):
    U = _extend_1d(U)                      # x first (last axis)
    bottom = U[..., :1, :].repeat_interleave(EXT, dim=-2)
    top = U[..., -1:, :].repeat_interleave(EXT, dim=-2)
    return torch.cat([bottom, U, top], dim=-2)   # corners: copies of the corner cells


def _state(dim, nx, ny, seed):
    if dim == 1:
        U = torch.tensor(fi.smooth_euler_1d(nx))
    else:
        U = torch.tensor(fi.random_euler_state_2d(nx, ny, seed, amp=0.2))
    return U


def _pair(dim, k, nx, ny, seed):
    U = _state(dim, nx, ny, seed)
    if dim == 1:
        dx = 2.0 / nx
        tr = S.Config(dim=1, nx=nx, x0=0.0, x1=2.0, k=k, system="euler", oe="off", bc_x="transmissive")
        pe = S.Config(dim=1, nx=nx + 2 * EXT, x0=-EXT * dx, x1=2.0 + EXT * dx, k=k, system="euler", oe="off",
                      bc_x="periodic")
        R_tr = S.residual(U, tr)
        R_pe = S.residual(_extend_1d(U), pe)[..., EXT:-EXT]
    else:
        dx, dy = 1.0 / nx, 1.0 / ny
        tr = S.Config(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, k=k, system="euler", oe="off",
                      bc_x="transmissive", bc_y="transmissive")
        pe = S.Config(dim=2, nx=nx + 2 * EXT, ny=ny + 2 * EXT, x0=-EXT * dx, x1=1.0 + EXT * dx,
                      y0=-EXT * dy, y1=1.0 + EXT * dy, k=k, system="euler", oe="off",
                      bc_x="periodic", bc_y="periodic")
        R_tr = S.residual(U, tr)
        R_pe = S.residual(_extend_2d(U), pe)[..., EXT:-EXT, EXT:-EXT]
    scale = float(torch.max(torch.abs(R_tr)))
    return float(torch.max(torch.abs(R_tr - R_pe))) / scale


@pytest.mark.parametrize("dim,k", [(1, 3), (1, 5), (2, 3), (2, 5), (2, 6)])
def test_transmissive_ghosts_act_as_copied_cells(dim, k):
    assert _pair(dim, k, 12, 9, 4) < 1e-14


def _second_cell(n, g, bc):
    idx = torch.arange(-g, n + g)
    if bc == "periodic":
        return idx % n
    return torch.where(idx < 0, torch.ones_like(idx), torch.where(idx >= n, torch.full_like(idx, n - 2), idx))


_orig_pad = S.pad


def _zero_ghost_moments(U, cfg, g=2, t=0.0):
    P = _orig_pad(U, cfg, g, t).clone()
    if cfg.bc_x == "transmissive":
        P[:, 1:, ..., :g] = 0.0
        P[:, 1:, ..., -g:] = 0.0
    return P


def _swapped_rules(U, cfg, g=2, t=0.0):
    if cfg.dim == 1 or cfg.bc_x == cfg.bc_y:
        # a rule that reads bc_x for the y-direction: here, periodic in y where transmissive is asked
        c = S.Config(**{**cfg.__dict__, "bc_y": "periodic" if cfg.bc_y == "transmissive" else cfg.bc_y}) \
            if cfg.dim == 2 else cfg
        return _orig_pad(U, c, g, t)
    return _orig_pad(U, cfg, g, t)


@pytest.mark.parametrize("plant", ["second_cell", "zero_moments", "swapped"])
def test_planted_ghost_mistakes_fail(plant, monkeypatch):
    if plant == "second_cell":
        monkeypatch.setattr(S, "_ghost_index", _second_cell)
    elif plant == "zero_moments":
        monkeypatch.setattr(S, "pad", _zero_ghost_moments)
    else:
        monkeypatch.setattr(S, "pad", _swapped_rules)
    worst = max(_pair(2, 5, 12, 9, 4), _pair(1, 5, 12, 9, 4) if plant != "swapped" else 0.0)
    assert worst > 1e-6
