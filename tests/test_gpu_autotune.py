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
    assert (hs == 0 or 8 <= hs <= 187) and 8 <= ho <= 187
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


@pytest.mark.parametrize("n", [(1000, 900), (2048, 2048)])
def test_tiling_choices_are_bitwise_neutral(n):
    """Fixed strip-tile heights and the limiter's cost-partitioned segment list (which
    re-cuts the strips after every stage launch from the recorded row costs) give the
    same state, bit for bit."""
    from paper_2609_26194_amd import Fam
    nx, ny = n
    _, cfg = both_configs(dim=2, nx=nx, ny=ny, k=5, system="euler", bc_x="transmissive",
                          bc_y="transmissive", oe="type2", cfl=0.2, pp=True)
    U0 = to_dev(fi.four_quadrant(nx, 0, ny=ny))
    outs = []
    for hs, ho in ((16, 16), (0, 40), (40, 24), (0, 8)):
        fam = Fam(cfg)
        fam.set_tiling(hs, ho)
        U = U0.clone()
        fam.run(U, 0.0, 4)
        fam.check()
        outs.append(U)
        log(f"  {nx}x{ny} stage H {hs} (0 = segment list), OE H {ho}: done")
        fam.close()
    for U in outs[1:]:
        assert torch.equal(U, outs[0])


def test_set_tiling_rejects_invalid_shapes():
    from paper_2609_26194_amd import Fam, FamConfig
    from paper_2609_26194_amd.fam import FamError
    plain = Fam(FamConfig(dim=2, nx=128, ny=96, k=5, system="euler", oe="type2"))
    with pytest.raises(FamError):
        plain.set_tiling(0, 16)          # segment list needs the limiter
    plain.set_tiling(96, 8)
    for bad in ((7, 16), (97, 16), (16, 0), (16, 97)):
        with pytest.raises(FamError):
            plain.set_tiling(*bad)
    batch = Fam(None, batch=[FamConfig(dim=2, nx=64, ny=64, k=5, system="euler")] * 2)
    with pytest.raises(FamError):
        batch.set_tiling(16, 16)
