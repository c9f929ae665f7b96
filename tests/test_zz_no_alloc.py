"""fam_step_static, the allocation-free step, against fam_step through the C ABI.

fam_step_static runs the kernels of fam_step with its scratch in a file-scope
device array instead of a context's allocations, so on the same input its result
must equal a fresh context's fam_step bit for bit.  Every case makes two calls in
a row, the second on a smaller mesh (the array keeps the first call's contents),
and also checks the second call against the oracle.  The cases cover the
positivity limiter's tile order, the Type I reductions, 1D, and the double Mach
reflection boundaries at a nonzero start time (the time argument).
"""
import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import both_configs, log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]


def _context_step(cfg, U0, t0):
    from paper_2609_26194_amd import Fam
    fam = Fam(cfg)
    U = to_dev(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    if t0:
        fam.set_time(t0)
    fam.step(U, 0.0, dt)
    fam.check()
    torch.cuda.synchronize()
    fam.close()
    return U, dt


def _static_step(cfg, U0, t0):
    from paper_2609_26194_amd.fam import fam_step_static
    U = to_dev(U0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    fam_step_static(cfg, stream.cuda_stream, U, t0, 0.0, dt, flag)
    torch.cuda.synchronize()
    assert int(flag[0]) == 0
    return U, dt


def _cases():
    big2d = dict(dim=2, nx=300, ny=250, k=5, system="euler", bc_x="transmissive", bc_y="transmissive", oe="type2",
                 cfl=0.2, pp=True)
    small2d = dict(dim=2, nx=70, ny=45, k=6, system="euler", bc_x="transmissive", bc_y="transmissive",
                   oe="type1", cfl=0.2, pp=True)
    big1d = dict(dim=1, nx=4000, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive", oe="type2", cfl=0.2)
    small1d = dict(dim=1, nx=200, x0=0.0, x1=6.283185307179586, k=3, system="advection", oe="type2", cfl=0.2)
    dmr_big = dict(dim=2, nx=240, ny=80, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2", cfl=0.2,
                   pp=True, dmr=True)
    dmr_small = dict(dmr_big, nx=96, ny=32)
    return {
        "2d_limiter_then_type1": ((big2d, fi.four_quadrant(300, 0, ny=250), 0.0),
                                  (small2d, fi.four_quadrant(70, 5, ny=45), 0.0)),
        "1d_euler_then_advection": ((big1d, fi.shu_osher(4000), 0.0), (small1d, fi.sine_advection(200), 0.0)),
        "double_mach_at_t": ((dmr_big, fi.double_mach(240, 80), 0.013), (dmr_small, fi.double_mach(96, 32), 0.021)),
    }


@pytest.mark.parametrize("case", ["2d_limiter_then_type1", "1d_euler_then_advection", "double_mach_at_t"])
def test_static_step_equals_fam_step_on_two_calls(case):
    for i, (kw, U0, t0) in enumerate(_cases()[case]):
        ora, cfg = both_configs(**kw)
        log(f"fam_step_static {case}, call {i + 1}: {kw['nx']}x{kw.get('ny', 1)} k={kw['k']} t0={t0}")
        Us, dts = _static_step(cfg, U0, t0)
        Uc, dtc = _context_step(cfg, U0, t0)
        assert torch.equal(dts, dtc), (float(dts[0]), float(dtc[0]))
        assert torch.equal(Us, Uc)
        ref, dt_ref = S.step(torch.tensor(U0), ora, t=t0)
        err = rel_linf(Us, ref)
        log(f"  bitwise equal to fam_step; dt {float(dts[0]):.6e} (oracle {dt_ref:.6e}); rel Linf vs oracle "
            f"{err:.2e}")
        assert abs(float(dts[0]) - dt_ref) <= 1e-14 * dt_ref and err <= 1e-12
