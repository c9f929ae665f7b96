"""fam_step allocates nothing and enqueues only kernels and device-to-device copies,
so a caller can capture it in a HIP graph.  Each case captures one step on the
context's stream, replays the graph three times with unrelated eager work and
synchronisations between the replays, and checks every replay bit for bit against
the same sequence of eager steps (and the time step each reports)."""
import pytest
import torch

import fam_inputs as fi
from gpu_util import log, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]


def _cases():
    from paper_2609_26194_amd import FamConfig
    return {
        "2d_limiter_segment_list": (FamConfig(dim=2, nx=130, ny=100, k=5, system="euler", bc_x="transmissive",
                                              bc_y="transmissive", oe="type2", cfl=0.2, pp=True),
                                    fi.four_quadrant(130, 3, ny=100), (0, 24)),
        "2d_limiter_fixed_tiles": (FamConfig(dim=2, nx=130, ny=100, k=5, system="euler", bc_x="transmissive",
                                             bc_y="transmissive", oe="type2", cfl=0.2, pp=True),
                                   fi.four_quadrant(130, 3, ny=100), (16, 16)),
        "2d_periodic_k6": (FamConfig(dim=2, nx=96, ny=64, k=6, system="euler", oe="type2", cfl=0.2),
                           fi.random_euler_state_2d(96, 64, 4, amp=0.1), None),
        "1d_shu_osher": (FamConfig(dim=1, nx=600, x0=-5.0, x1=5.0, k=5, system="euler", bc_x="transmissive",
                                   oe="type2", cfl=0.2), fi.shu_osher(600), None),
    }


@pytest.mark.parametrize("case", ["2d_limiter_segment_list", "2d_limiter_fixed_tiles", "2d_periodic_k6",
                                  "1d_shu_osher"])
def test_captured_step_replays_match_eager_steps(case):
    from paper_2609_26194_amd import Fam
    cfg, U0h, tiling = _cases()[case]
    log(f"graph-captured fam_step: {case}")
    fam = Fam(cfg)
    if tiling is not None:
        fam.set_tiling(*tiling)
    U0 = to_dev(U0h)
    # eager reference: three steps
    Ue = U0.clone()
    dte = torch.empty(1, dtype=torch.float64, device="cuda")
    refs = []
    for _ in range(3):
        fam.step(Ue, 0.0, dte)
        refs.append((Ue.clone(), dte.clone()))
    torch.cuda.synchronize()
    # capture one step on the context's stream
    Ug = U0.clone()
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=fam.stream):
        fam.step(Ug, 0.0, dtg)
    torch.cuda.synchronize()
    assert torch.equal(Ug, U0)   # capturing runs nothing
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ug, refs[r][0]), f"replay {r}"
        assert torch.equal(dtg, refs[r][1])
        # unrelated eager work between replays
        junk = torch.randn(4096, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        del junk
    fam.check()
    log(f"  3 replays bitwise equal to the eager steps (dt {float(dtg[0]):.6e})")
    del g
    fam.close()
