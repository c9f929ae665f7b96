"""The paper's smooth accuracy tables reproduced on the GPU (Sec. 4: Tables 1dBur,
1dEuler, 2dEuler; OE Type II, C = 0.1, time step C dx^{k/3} / alpha, i.e. dt_rule = 1).

Errors are the mean absolute error of the density (Burgers: u) cell averages
against the exact cell averages at the final time; the printed values are the
paper's (tests/golden/smooth_accuracy_tables.txt).  They are compared within the
same factors as the oracle's own pins (Euler's averages sit 1.4-2x above the
printed values for a reason not identified, while the first moments of the same
runs match closely; Burgers FAM4 differs most) at every printed mesh size, the
upper bound raised to the accumulated FP64 rounding of the run (steps x 2^-52 x
max|u|) where FAM6 on the finest meshes reaches it.  The 2D table runs N = 20..80
by default and 100, 120 with FAM_SLOW=1.  One run per system is
also compared with the oracle step for step (the whole time-step sequence,
including the dx^{k/3} rule and the clipped last step).

The appendix tables of first-moment errors (supp:1dBurMoment, supp:1dEulerMoment)
are reproduced at every printed mesh size: the mean absolute error of the scaled
first moment of the density (Burgers: u) within per-order factors of the printed
value, and the observed order over the whole range of at least k - 0.5.
"""

# the factor within which the first-moment errors reproduce the printed ones
MOM_TOL = {3: 1.5, 4: 2.0, 5: 1.5, 6: 1.5}
EPS = 2.0 ** -52


def _rounding_floor(steps, umax):
    """Accumulated FP64 rounding of a run: below steps * eps * max|u| an error cannot be told
    from the printed one (FAM6 on the finest meshes reaches it after 5e4 - 3e5 steps)."""
    return steps * EPS * umax


def _check_avg(name, n, k, e, steps, tol, umax):
    g = _gold(name, n, k)
    hi = max(g * tol, _rounding_floor(steps, umax))
    log(f"  {name} FAM{k} N={n}: {steps} steps, error {e:.3e} (printed {g:.3e}, ratio {e / g:.3f}, "
        f"bound {hi:.2e})")
    assert g / tol < e < hi
import math
import os

import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from golden_util import parse_table
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
GOLD = parse_table("smooth_accuracy_tables.txt")


def _gold(table, n, k):
    for name, nn, vals in GOLD:
        if name == table and nn == n:
            return vals[k - 3]
    raise KeyError((table, n))


def _fam(cfg):
    from paper_2609_26194_amd import Fam
    return Fam(cfg)


def _run(cfg, U0, T):
    fam = _fam(cfg)
    U = to_dev(U0)
    steps, t = fam.run(U, T, 10 ** 7)
    fam.check()
    assert abs(t - T) <= 1e-14 * max(1.0, T)
    return U.cpu().numpy(), steps


@pytest.mark.parametrize("k,tol", [(3, 1.6), (4, 1.8), (5, 1.15), (6, 1.15)])
def test_burgers_table(k, tol):
    T = 0.5 / math.pi
    errs = []
    for n in (30, 60, 90, 120, 150, 180):
        _, cfg = both_configs(dim=1, nx=n, x0=0.0, x1=2.0, k=k, system="burgers", oe="type2", cfl=0.1,
                              dt_rule=1)
        U, steps = _run(cfg, fi.burgers_smooth(n), T)
        e = float(np.abs(U[0, 0] - fi.burgers_exact_moments(n, T)[0, 0]).mean())
        _check_avg("burgers_avg", n, k, e, steps, tol, 1.5)
        errs.append(e)
    order = math.log(errs[1] / errs[2]) / math.log(90 / 60)
    log(f"  order 60 -> 90: {order:.2f}")
    assert order > k + 1 - 0.6


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_euler_1d_table(k):
    for n in (20, 30, 40, 50, 60, 70):
        _, cfg = both_configs(dim=1, nx=n, x0=0.0, x1=2.0, k=k, system="euler", oe="type2", cfl=0.1, dt_rule=1)
        U, steps = _run(cfg, fi.smooth_euler_1d(n), 2.0)
        e = float(np.abs(U[0, 0] - fi.smooth_euler_1d_exact_density(n, 2.0)[0, 0]).mean())
        _check_avg("euler1d_avg", n, k, e, steps, 2.5, 1.2)


EULER2D_N = (20, 40, 60, 80) + ((100, 120) if os.environ.get("FAM_SLOW") == "1" else ())


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_euler_2d_table(k):
    """N = 20..80 by default; the 100 and 120 rows (3e5 steps at FAM6) with FAM_SLOW=1."""
    for n in EULER2D_N:
        _, cfg = both_configs(dim=2, nx=n, ny=n, x0=0.0, x1=2.0, y0=0.0, y1=2.0, k=k, system="euler", oe="type2",
                              cfl=0.1, dt_rule=1)
        U, steps = _run(cfg, fi.smooth_euler_2d(n), 2.0)
        e = float(np.abs(U[0, 0] - fi.smooth_euler_2d_exact_density(n, 2.0)[0, 0]).mean())
        _check_avg("euler2d_avg", n, k, e, steps, 3.0, 1.2)


@pytest.mark.parametrize("system,dim", [("burgers", 1), ("euler", 1), ("euler", 2)])
def test_smooth_rule_runs_match_the_oracle(system, dim):
    """The dx^{k/3} time-step rule and the clipped last step, against the oracle's run."""
    k, n = 5, 24
    if dim == 1:
        ora, cfg = both_configs(dim=1, nx=n, x0=0.0, x1=2.0, k=k, system=system, oe="type2", cfl=0.1, dt_rule=1)
        U0 = fi.burgers_smooth(n) if system == "burgers" else fi.smooth_euler_1d(n)
        T = 0.1
    else:
        ora, cfg = both_configs(dim=2, nx=n, ny=n, x0=0.0, x1=2.0, y0=0.0, y1=2.0, k=k, system="euler",
                                oe="type2", cfl=0.1, dt_rule=1)
        U0 = fi.smooth_euler_2d(n)
        T = 0.05
    ref, t_ref, steps_ref = S.run(torch.tensor(U0), ora, t_final=T)
    fam = _fam(cfg)
    U = to_dev(U0)
    steps, t = fam.run(U, T, 10 ** 6)
    log(f"  {system} {dim}D: {steps} steps (oracle {steps_ref}), t {t} (oracle {t_ref})")
    assert steps == steps_ref and abs(t - t_ref) <= 1e-15 * T
    err = rel_linf(U, ref)
    log(f"  rel Linf {err:.3e}")
    assert err <= 1e-12


def _moment_table(table, k, ns, make, exact, T):
    errs = []
    for n in ns:
        _, cfg = both_configs(dim=1, nx=n, x0=0.0, x1=2.0, k=k, system="burgers" if table == "burgers_mom" else "euler",
                              oe="type2", cfl=0.1, dt_rule=1)
        U, steps = _run(cfg, make(n), T)
        e = float(np.abs(U[0, 1] - exact(n, T)[0, 1]).mean())
        g = _gold(table, n, k)
        log(f"  {table} FAM{k} N={n}: {steps} steps, first-moment error {e:.3e} (printed {g:.3e}, ratio {e / g:.3f})")
        assert g / MOM_TOL[k] < e < g * MOM_TOL[k]
        errs.append(e)
    order = math.log(errs[0] / errs[-1]) / math.log(ns[-1] / ns[0])
    log(f"  order {ns[0]} -> {ns[-1]}: {order:.2f}")
    assert order > k - 0.5


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_burgers_moment_table(k):
    _moment_table("burgers_mom", k, (30, 60, 90, 120, 150, 180), fi.burgers_smooth, fi.burgers_exact_moments,
                  0.5 / math.pi)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_euler_1d_moment_table(k):
    _moment_table("euler1d_mom", k, (20, 30, 40, 50, 60, 70), fi.smooth_euler_1d, fi.smooth_euler_1d_exact_density,
                  2.0)
