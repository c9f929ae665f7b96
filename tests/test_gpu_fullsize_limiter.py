"""Full-size steps with the positivity limiter, in the launch configuration the
benchmark times, against stored oracle samples (tests/golden/fullsize_limiter_one_step.npz,
written by tests/golden/make_fullsize_limiter_samples.py from the oracle only).

* 2048 x 2048 four-quadrant data (seed 0), k = 5 and 6, OE Type II, limiter: the tilings the
  autotuner picks (as bench.py does) and the segment list, one step each.
* The double Mach reflection at the paper's size, 1440 x 480, k = 5, limiter, from t = 0.

* The batched workload (256 instances, sizes from seed 1, data seeds 1000 + i, limiter),
  autotuned as the benchmark runs it, one step: the first instance of each of the seven sizes
  against the oracle's step of that instance (every cell).

The samples hold the boundary rows and columns, the discontinuities of the initial
data, random cells and up to 256 cells whose stage-0 reconstruction the oracle's
limiter scales.  Bar: the time step to 1e-14 and every sampled moment within 1e-12 of
the component's largest average.
"""
import os

import numpy as np
import pytest
import torch

import fam_inputs as fi
import oracle.scheme as S
from gpu_util import log, needs_gpu, rel_linf, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]
TOL = 1e-12
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_limiter_one_step.npz")


def _check(fam, U, gold, prefix):
    cells = gold[prefix + "cells_ji"]
    dtd = fam.dt(U)
    dt_ref = float(gold[prefix + "dt"][0])
    assert abs(float(dtd[0]) - dt_ref) <= 1e-14 * dt_ref
    fam.run(U, 0.0, 1)
    fam.check()
    ji = [torch.as_tensor(cells[:, 0]).cuda(), torch.as_tensor(cells[:, 1]).cuda()]
    got = U[:, :, ji[0], ji[1]].cpu().numpy()
    ref, scale = gold[prefix + "values"], gold[prefix + "avg_absmax"]
    err = max(float(np.max(np.abs(got[c] - ref[c]))) / float(scale[c]) for c in range(4))
    log(f"  {len(cells)} sampled cells ({int(gold[prefix + 'n_limited_stage0'][0])} limited at stage 0 in the oracle):"
        f" rel Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("tiling", ["autotuned", "segment_list"])
@pytest.mark.parametrize("k", [5, 6])
def test_four_quadrant_2048_with_limiter(k, tiling):
    from paper_2609_26194_amd import Fam, FamConfig
    gold = np.load(GOLD)
    log(f"four-quadrant 2048^2 k={k} limiter, {tiling}")
    cfg = FamConfig(dim=2, nx=2048, ny=2048, k=k, system="euler", bc_x="transmissive", bc_y="transmissive",
                    oe="type2", cfl=0.2, pp=True)
    U0 = to_dev(fi.four_quadrant(2048, 0))
    fam = Fam(cfg)
    if tiling == "autotuned":
        log(f"  autotuned tile heights {fam.autotune(U0)}")
    else:
        fam.set_tiling(0, 36)
    _check(fam, U0.clone(), gold, "c3pp_" if k == 5 else "c3pp6_")
    fam.close()


def test_double_mach_1440x480_with_limiter():
    from paper_2609_26194_amd import Fam, FamConfig
    gold = np.load(GOLD)
    log("double Mach reflection 1440x480 k=5 limiter, autotuned")
    cfg = FamConfig(dim=2, nx=1440, ny=480, x0=0.0, x1=3.0, y0=0.0, y1=1.0, k=5, system="euler", oe="type2",
                    cfl=0.2, pp=True, dmr=True)
    U0 = to_dev(fi.double_mach(1440, 480))
    fam = Fam(cfg)
    log(f"  autotuned tile heights {fam.autotune(U0)}")
    _check(fam, U0.clone(), gold, "dmr_")
    fam.close()


def test_batched_256_instances_with_limiter():
    from paper_2609_26194_amd import Fam, FamConfig
    sizes = fi.batch_sizes(256, 1)
    kw = dict(dim=2, k=5, system="euler", bc_x="transmissive", bc_y="transmissive", oe="type2", cfl=0.2, pp=True)
    cfgs = [FamConfig(nx=n, ny=n, **kw) for n in sizes]
    states = [fi.batch_instance(i, n) for i, n in enumerate(sizes)]
    bat = Fam(cfgs[0], batch=cfgs)
    offs = bat.offsets()
    U0 = torch.zeros(bat.len, dtype=torch.float64, device="cuda")
    for o, st in zip(offs, states):
        U0[o:o + st.size] = torch.as_tensor(st.reshape(-1)).cuda()
    log(f"batched 256 instances ({sum(n * n for n in sizes)} cells), autotuned {bat.autotune(U0)}")
    U = U0.clone()
    bat.run(U, 0.0, 1)
    bat.check()
    firsts = {}
    for i, n in enumerate(sizes):
        firsts.setdefault(n, i)
    for n, i in sorted(firsts.items()):
        ref, _ = S.step(torch.tensor(states[i]), S.Config(nx=n, ny=n, **kw))
        got = U[offs[i]:offs[i] + states[i].size].reshape(states[i].shape)
        err = rel_linf(got, ref)
        log(f"  instance {i} ({n}x{n}): rel Linf {err:.3e}")
        assert err <= TOL
    bat.close()
