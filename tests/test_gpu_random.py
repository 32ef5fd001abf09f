"""Randomized GPU parity: seeded random shapes (ragged, partial tiles), boundaries per
axis, Hamiltonian families and parameters, and schemes.  One step through the C ABI
against the FP64 oracle: FP64 within 1e-12 of max|phi|, the FP32 stencil within 2e-6."""
import os

import numpy as np
import pytest

import oracle as O
import random_configs as RC
from paper_1909_13263_amd import hjw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    assert os.path.dirname(hjw.LIB_PATH).endswith("paper_1909_13263_amd")
    yield


@pytest.mark.parametrize("seed", range(40))
def test_random_configuration_one_step(seed):
    cfg = RC.random_config(seed)
    dim = len(cfg["shape"])
    bcs = cfg["bcs"] if dim == 2 else (cfg["bcs"][0], cfg["bcs"][0])
    prob = O.Problem(cfg["shape"], RC.spacing(cfg), cfg["ham"], cfg["params"], bcs,
                     scheme=cfg["scheme"], origin=RC.origin(cfg))
    ref, info = O.rk3_step(prob, cfg["phi"], 0.0, 1.0, 0.5)
    scale = np.abs(ref).max()
    for prec, tol in [(hjw.FP64, 1e-12), (hjw.FP32_MIXED, 2e-6)]:
        g = hjw.Grid(cfg["shape"], cfg["lo"], cfg["hi"], cfg["bcs"] if dim == 2 else cfg["bcs"][0],
                     prec)
        g.set_hamiltonian(cfg["ham"], cfg["params"])
        if cfg["scheme"]:
            g.set_scheme(cfg["scheme"])
        g.set_phi(cfg["phi"])
        gi = g.step_to(1.0, 0.5, max_steps=1)
        phi = g.get_phi()
        g.close()
        assert gi.steps == 1
        err = float(np.abs(phi - ref).max() / scale)
        assert err <= tol, (seed, prec, err, cfg["shape"], cfg["ham"], cfg["bcs"])
