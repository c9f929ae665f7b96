"""The launch-shape autotuner changes how the work is tiled, never the result."""
import pytest
import torch

import fam_inputs as fi
from gpu_util import both_configs, log, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_autotune_single_is_bitwise_neutral():
    from paper_2609_26194_amd import Fam
    _, cfg = both_configs(dim=2, nx=301, ny=187, k=5, system="euler", bc_x="transmissive",
                          bc_y="transmissive", oe="type2", cfl=0.2, pp=True)
    U0 = to_dev(fi.four_quadrant(301, 0, ny=187))
    ref = Fam(cfg)
    Ur = U0.clone()
    ref.run(Ur, 0.0, 6)
    fam = Fam(cfg)
    hs, ho = fam.autotune(U0, reps=2)
    log(f"autotune 301x187: stage H {hs}, OE H {ho}")
    assert hs in (8, 12, 16, 20, 24, 28, 32, 40, 48, 64) and ho in (8, 12, 16, 20, 24, 28, 32, 40, 48, 64)
    U = U0.clone()
    fam.run(U, 0.0, 6)
    fam.check()
    assert torch.equal(U, Ur)


def test_autotune_batched_is_bitwise_neutral():
    from paper_2609_26194_amd import Fam, FamConfig
    sizes = [64, 96, 130, 62, 200, 75]
    cfgs = [FamConfig(dim=2, nx=n, ny=n, k=5, system="euler", bc_x="transmissive", bc_y="transmissive",
                      oe="type2", cfl=0.2, pp=True) for n in sizes]
    states = [fi.batch_instance(i, n) for i, n in enumerate(sizes)]
    outs = []
    for tune in (False, True):
        bat = Fam(cfgs[0], batch=cfgs)
        Ub = torch.zeros(bat.len, dtype=torch.float64, device="cuda")
        for o, s in zip(bat.offsets(), states):
            Ub[o:o + s.size] = to_dev(s).reshape(-1)
        if tune:
            h, p = bat.autotune(Ub, reps=2)
            log(f"autotune batch: H {h}, persistent blocks {p}")
        bat.run(Ub, 0.0, 5)
        bat.check()
        outs.append(Ub)
    assert torch.equal(outs[0], outs[1])
