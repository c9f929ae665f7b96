"""Checks of the oracle's reference gradient (used to pin the HIP adjoint).

The reference gradient is reverse-mode differentiation of the oracle's own FAM
steps.  It is checked here against things outside torch's reverse mode: central
finite differences of the oracle's forward map, and forward-mode (dual-number)
directional derivatives.

Non-differentiable points.  The OE coefficient of a system is a maximum over
components (eq. 2dOE_system).  On the density-wave state (u = v = 1/2, p = 1) the
momenta are exactly rho/2, so the components rho, rho u, rho v have identical
jump ratios and the maximum ties: J is not differentiable there with OE on, and
a central difference along an arbitrary direction returns the mean of the two
one-sided derivatives.  Along directions that keep u, v and p fixed the tie
persists and J is differentiable; those are the directions used on that state.
Generic directions are used with OE off and on a state without ties.
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
from oracle.functional import directional_derivative, functional, reference_gradient, run_fixed
from oracle.scheme import Config, cfl_dt


def _states():
    return {
        "density_waves": lambda n: fi.density_waves(n),
        "tie_free": lambda n: fi.random_euler_state_2d(n, n, 4, amp=0.1),
    }


@pytest.mark.parametrize("oe,state,tie_preserving", [
    ("off", "density_waves", False),
    ("type2", "density_waves", True),
    ("type2", "tie_free", False),
    ("type1", "tie_free", False),
])
def test_reference_gradient_matches_finite_differences(oe, state, tie_preserving):
    n = 8
    cfg = Config(dim=2, nx=n, ny=n, k=5, system="euler", oe=oe)
    U0 = torch.tensor(_states()[state](n))
    dt = cfl_dt(U0, cfg)
    J, g = reference_gradient(U0, cfg, 2, dt)
    rng = np.random.default_rng(0)
    for _ in range(3):
        if tie_preserving:
            d = torch.tensor(fi.density_wave_direction(n, rng))
        else:
            d = torch.tensor(rng.standard_normal(U0.shape))
        # unit-norm direction, small step: stay clear of the |jump| kinks of the OE
        # (face jumps of this smooth state go down to ~2e-6)
        d = d / torch.linalg.norm(d)
        eps = 1e-6
        jp = float(functional(run_fixed(U0 + eps * d, cfg, 2, dt), cfg))
        jm = float(functional(run_fixed(U0 - eps * d, cfg, 2, dt), cfg))
        fd = (jp - jm) / (2 * eps)
        ad = float((g * d).sum())
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12, (fd, ad)
        dual = directional_derivative(U0, cfg, 2, dt, d)
        assert abs(dual - ad) <= 1e-12 * abs(ad) + 1e-15


def test_density_wave_state_has_tied_oe_components():
    """The kink described above is real: one-sided derivatives differ along a generic direction."""
    n = 8
    cfg = Config(dim=2, nx=n, ny=n, k=5, system="euler", oe="type2")
    U0 = torch.tensor(fi.density_waves(n))
    dt = cfl_dt(U0, cfg)
    J = float(functional(run_fixed(U0, cfg, 2, dt), cfg))
    d = torch.tensor(np.random.default_rng(0).standard_normal(U0.shape))
    eps = 1e-7
    fwd = (float(functional(run_fixed(U0 + eps * d, cfg, 2, dt), cfg)) - J) / eps
    bwd = (J - float(functional(run_fixed(U0 - eps * d, cfg, 2, dt), cfg))) / eps
    assert abs(fwd - bwd) > 1e-3 * abs(fwd)


def test_functional_of_a_constant_state():
    n = 8
    cfg = Config(dim=2, nx=n, ny=n, k=5, system="euler")
    U = torch.zeros(4, 3, n, n, dtype=torch.float64)
    U[0, 0] = 2.0
    # window [1/4, 3/4]^2 has area 1/4: J = 4 * 1/4
    assert abs(float(functional(U, cfg)) - 1.0) < 1e-15
