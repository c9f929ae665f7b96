"""Helpers shared by the GPU tests: config mapping and the parity metric."""
import numpy as np
import pytest
import torch

from oracle.scheme import Config

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")


def both_configs(**kw):
    """(oracle Config, library FamConfig) built from one set of keyword arguments."""
    from paper_2609_26194_amd import FamConfig
    ora = Config(**kw)
    return ora, FamConfig(**kw)


def to_dev(U):
    return torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64).cuda()


def rel_linf(gpu, ora):
    """max over components c of max|U_gpu - U_ora| / max|U_ora average of c|."""
    g = np.asarray(gpu.detach().cpu() if isinstance(gpu, torch.Tensor) else gpu, dtype=np.float64)
    o = np.asarray(ora.detach().cpu() if isinstance(ora, torch.Tensor) else ora, dtype=np.float64)
    assert g.shape == o.shape, (g.shape, o.shape)
    worst = 0.0
    for c in range(o.shape[0]):
        scale = max(float(np.max(np.abs(o[c, 0]))), 1e-300)
        worst = max(worst, float(np.max(np.abs(g[c] - o[c]))) / scale)
    return worst


def log(msg):
    print(msg, flush=True)
