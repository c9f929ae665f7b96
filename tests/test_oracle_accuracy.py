"""Accuracy pins of the oracle against the paper's convergence claims and printed errors.

* Prop. 3.3 (cell-average superconvergence of the linear backbone): on sine
  advection with OE off and dt ~ dx^{(k+1)/3} (so RK3's error does not mask the
  spatial one), averages converge with order k+1 and first moments with order k.
* Prop. 2.2(ii): the OE pass does not reduce the order (sine advection, OE Type II).
* Tables 1dBur and 1dEuler (smooth Burgers, smooth 1D Euler, OE Type II,
  C = 0.1, dt = C dx^{k/3}/alpha): errors of the density averages (mean absolute
  error over cells) within 1.2x of the printed values, under the reading that the
  printed runs used half the stated gamma_k (equivalently, the mean of the two
  interface jumps; golden_util.table_gamma_k).  The Burgers rows also pin the
  global Lax-Friedrichs reading of the numerical flux.
* The appendix tables of first-moment errors for the same two runs
  (supp:1dBurMoment, supp:1dEulerMoment): the scaled first moment of the same
  oracle states against the exact first moment, within 1.25x.
* Table 2dEuler, FAM3 at N = 20 under the same reading, within 1.2x (FAM5/FAM6 sit
  about 2x above their rows also with OE off: a known gap, measured on the GPU).
* The stated gamma_k (the library's default) against the tables: the 1D Euler FAM4
  error at N = 20 sits about 2.1x above the printed value, which the halved
  reading removes; this test records that the choice of reading matters.
"""

# the factor within which the oracle's errors reproduce the printed ones (table reading)
AVG_TOL = 1.2
MOM_TOL = 1.25
import math

import numpy as np
import pytest
import torch

import fam_inputs as fi
from golden_util import parse_table, table_gamma_k
from oracle.scheme import Config, run, step

GOLD = parse_table("smooth_accuracy_tables.txt")


def _sine_errors(k, n, dt_rule, oe):
    cfg = Config(dim=1, nx=n, k=k, system="advection", oe=oe, x0=0.0, x1=2 * math.pi)
    T = 2 * math.pi
    dt0 = dt_rule(cfg.dx)
    nsteps = int(math.ceil(T / dt0 - 1e-9))
    U, _, _ = run(torch.tensor(fi.sine_advection(n)), cfg, nsteps=nsteps, dt=T / nsteps)
    ex = fi.sine_advection(n)   # one period later the exact solution is the initial one
    e0 = np.abs(U[0, 0].numpy() - ex[0, 0]).mean()
    e1 = np.abs(U[0, 1].numpy() - ex[0, 1]).mean()
    return e0, e1


@pytest.mark.parametrize("k", [3, 4])
def test_cell_average_superconvergence(k):
    ns = (40, 80, 160)
    errs = [_sine_errors(k, n, lambda dx: 0.2 * dx ** ((k + 1) / 3), "off") for n in ns]
    o0 = math.log2(errs[1][0] / errs[2][0])
    o1 = math.log2(errs[1][1] / errs[2][1])
    assert o0 > k + 1 - 0.25, (k, errs)
    assert k - 0.3 < o1 < k + 0.6, (k, errs)


def test_oe_keeps_the_order_on_sine_advection():
    """Sine advection at dt = 0.2 dx (5N steps to t = 2 pi): FAM3 with OE Type II."""
    ns = (50, 100, 200)
    errs = [_sine_errors(3, n, lambda dx: 0.2 * dx, "type2") for n in ns]
    o0 = math.log2(errs[1][0] / errs[2][0])
    o1 = math.log2(errs[1][1] / errs[2][1])
    # averages: RK3's O(dt^3) error dominates at dt = 0.2 dx; moments: order k.
    # (The Type II denominator vanishes at the zero crossings of this data, so the
    # premise of Prop. 2.2(ii) fails locally; only the orders are asserted.)
    assert o0 > 2.9 and o1 > 2.8, errs


def _smooth_run(system, k, n, T, U0, gamma_k=None):
    x1 = 2.0
    cfg = Config(dim=1, nx=n, x0=0.0, x1=x1, k=k, system=system, oe="type2",
                 oe_gamma_k=table_gamma_k(1, k) if gamma_k is None else gamma_k)
    U = torch.tensor(U0)
    t = 0.0
    while t < T:
        alpha = float(torch.max(cfg.phys.speed(U[:, 0], 0)))
        dt = min(0.1 * cfg.dx ** (k / 3) / alpha, T - t)
        U, _ = step(U, cfg, dt)
        t += dt
    return U


def _gold(table, n, k):
    for name, nn, vals in GOLD:
        if name == table and nn == n:
            return vals[k - 3]
    raise KeyError((table, n))


@pytest.mark.parametrize("k,ns", [(3, (30, 60)), (4, (30, 60)), (5, (30, 60)), (6, (30, 60))])
def test_burgers_table(k, ns):
    """Every order at N = 30 and 60 (the GPU runs every printed N)."""
    T = 0.5 / math.pi
    for n in ns:
        U = _smooth_run("burgers", k, n, T, fi.burgers_smooth(n))
        ex = fi.burgers_exact_moments(n, T)
        e = np.abs(U[0, 0].numpy() - ex[0, 0]).mean()
        g = _gold("burgers_avg", n, k)
        assert g / AVG_TOL < e < g * AVG_TOL, (k, n, e, g)
        e1 = np.abs(U[0, 1].numpy() - ex[0, 1]).mean()
        g1 = _gold("burgers_mom", n, k)
        assert g1 / MOM_TOL < e1 < g1 * MOM_TOL, (k, n, e1, g1)


@pytest.mark.parametrize("k,ns", [(3, (20, 30)), (4, (20, 30)), (5, (20,)), (6, (20,))])
def test_euler_1d_table(k, ns):
    for n in ns:
        U = _smooth_run("euler", k, n, 2.0, fi.smooth_euler_1d(n))
        ex = fi.smooth_euler_1d_exact_density(n, 2.0)
        e = np.abs(U[0, 0].numpy() - ex[0, 0]).mean()
        g = _gold("euler1d_avg", n, k)
        assert g / AVG_TOL < e < g * AVG_TOL, (k, n, e, g)
        e1 = np.abs(U[0, 1].numpy() - ex[0, 1]).mean()
        g1 = _gold("euler1d_mom", n, k)
        assert g1 / MOM_TOL < e1 < g1 * MOM_TOL, (k, n, e1, g1)


def test_stated_gamma_k_misses_the_1d_euler_table():
    """At the text's gamma_4 = 25 the FAM4 error at N = 20 is about 2.1x the printed one;
    the halved reading brings it to 1.09x (test_euler_1d_table)."""
    n, k = 20, 4
    U = _smooth_run("euler", k, n, 2.0, fi.smooth_euler_1d(n), gamma_k=25.0)
    e = np.abs(U[0, 0].numpy() - fi.smooth_euler_1d_exact_density(n, 2.0)[0, 0]).mean()
    assert 1.9 < e / _gold("euler1d_avg", n, k) < 2.3


def _euler_2d(n, k, oe="type2"):
    cfg = Config(dim=2, nx=n, ny=n, x0=0, x1=2, y0=0, y1=2, k=k, system="euler", oe=oe,
                 oe_gamma_k=table_gamma_k(2, k))
    U = torch.tensor(fi.smooth_euler_2d(n))
    t, T = 0.0, 2.0
    while t < T:
        ax = float(torch.max(cfg.phys.speed(U[:, 0], 0)))
        ay = float(torch.max(cfg.phys.speed(U[:, 0], 1)))
        dt = min(0.1 / (ax / cfg.dx ** (k / 3) + ay / cfg.dy ** (k / 3)), T - t)
        U, _ = step(U, cfg, dt)
        t += dt
    return np.abs(U[0, 0].numpy() - fi.smooth_euler_2d_exact_density(n, T)[0, 0]).mean()


def test_euler_2d_table_fam3():
    """Table 2dEuler, FAM3 at N = 20, within 1.2x under the table reading.  (FAM5/FAM6 sit
    about 2x above their printed values also with OE off, a known gap; the GPU runs
    every printed row and states the ratios.)"""
    n, k = 20, 3
    g = _gold("euler2d_avg", n, k)
    assert 1 / AVG_TOL < _euler_2d(n, k) / g < AVG_TOL
