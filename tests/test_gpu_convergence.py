"""Convergence of 1D sine advection on the GPU (u_t + u_x = 0 on periodic [0, 2 pi],
u0 = sin x + cos(3x)/2, FAM3, dt = 0.2 dx, one period: 5N steps), N = 50 .. 800.

* OE off: the fully discrete linear scheme has the closed form U^n = G(xi)^n u_ex per
  Fourier mode (Sec. 3: the printed D matrices, the SSP-RK3 amplification matrix
  and the printed exact moment vector), so every N is compared with it directly.
  The orders follow: first moments k = 3, averages above 3 (the averages' spatial
  superconvergence is masked by RK3's O(dt^3) at dt = 0.2 dx).
* OE Type II (Prop. 2.2(ii)): the order is kept (averages and moments at least 2.9
  and 2.8 between consecutive meshes), and at every N the first steps match the
  oracle to 1e-12.
"""
import math

import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev
from test_oracle_fourier import closed_form_sine_advection

pytestmark = [pytest.mark.gpu, needs_gpu]
NS = (50, 100, 200, 400, 800)
T = 2 * math.pi


def _run(n, oe):
    ora, cfg = both_configs(dim=1, nx=n, x0=0.0, x1=T, k=3, system="advection", oe=oe, cfl=0.2)
    from paper_2609_26194_amd import Fam
    fam = Fam(cfg)
    U0 = fi.sine_advection(n)
    nsteps = 5 * n
    U = to_dev(U0)
    steps, _ = fam.run(U, 0.0, nsteps, T / nsteps)
    fam.check()
    assert steps == nsteps
    return ora, fam, U0, U.cpu().numpy(), nsteps


def _orders(errs):
    return [math.log2(a / b) for a, b in zip(errs, errs[1:])]


def test_sine_advection_convergence_oe_off_equals_the_closed_form():
    e0, e1 = [], []
    for n in NS:
        _, fam, U0, U, nsteps = _run(n, "off")
        fam.close()
        ref = closed_form_sine_advection(3, n, nsteps, 0.2)
        dev = float(np.max(np.abs(U[0] - ref)))
        ex = fi.sine_advection(n)[0]
        e0.append(float(np.abs(U[0, 0] - ex[0]).mean()))
        e1.append(float(np.abs(U[0, 1] - ex[1]).mean()))
        log(f"  N={n}: {nsteps} steps, |GPU - G(xi)^n u_ex| = {dev:.2e}; errors {e0[-1]:.3e} / {e1[-1]:.3e}")
        assert dev <= 1e-12
    o0, o1 = _orders(e0), _orders(e1)
    log(f"  orders: averages {['%.2f' % o for o in o0]}, first moments {['%.2f' % o for o in o1]}")
    assert min(o0) > 2.95 and all(2.8 < o < 3.3 for o in o1)


def test_sine_advection_convergence_with_oe_type2():
    e0, e1 = [], []
    for n in NS:
        ora, fam, U0, U, nsteps = _run(n, "type2")
        # the first steps against the oracle, same launch path
        ref5, _, _ = S.run(torch.tensor(U0), ora, nsteps=5, dt=T / nsteps)
        U5 = to_dev(U0)
        fam.run(U5, 0.0, 5, T / nsteps)
        err = rel_linf(U5, ref5)
        fam.close()
        ex = fi.sine_advection(n)[0]
        e0.append(float(np.abs(U[0, 0] - ex[0]).mean()))
        e1.append(float(np.abs(U[0, 1] - ex[1]).mean()))
        log(f"  N={n}: errors {e0[-1]:.3e} / {e1[-1]:.3e}; 5 steps vs oracle {err:.2e}")
        assert err <= 1e-12
    o0, o1 = _orders(e0), _orders(e1)
    log(f"  orders: averages {['%.2f' % o for o in o0]}, first moments {['%.2f' % o for o in o1]}")
    assert min(o0) > 2.9 and min(o1) > 2.8
