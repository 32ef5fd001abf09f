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


@pytest.mark.parametrize("seed", range(20))
def test_random_timed_configuration_three_steps(seed):
    """H(x, t, phi, D phi) with random shapes, boundaries, (a, b, w, lam) and schemes: three
    steps (the later ones at t_n > 0) against the oracle."""
    cfg = RC.random_timed_config(seed)
    dim = len(cfg["shape"])
    bcs = cfg["bcs"] if dim == 2 else (cfg["bcs"][0], cfg["bcs"][0])
    prob = O.Problem(cfg["shape"], RC.spacing(cfg), cfg["ham"], cfg["params"], bcs,
                     scheme=cfg["scheme"])
    ref, info = O.step_to(prob, cfg["phi"], 1.0, 0.5, max_steps=3)
    scale = np.abs(ref).max()
    for prec, tol in [(hjw.FP64, 1e-12), (hjw.FP32_MIXED, 2e-6)]:
        g = hjw.Grid(cfg["shape"], cfg["lo"], cfg["hi"], cfg["bcs"] if dim == 2 else cfg["bcs"][0],
                     prec)
        g.set_hamiltonian(cfg["ham"], cfg["params"])
        if cfg["scheme"]:
            g.set_scheme(cfg["scheme"])
        g.set_phi(cfg["phi"])
        gi = g.step_to(1.0, 0.5, max_steps=3)
        phi = g.get_phi()
        g.close()
        assert gi.steps == info.steps
        err = float(np.abs(phi - ref).max() / scale)
        assert err <= tol, (seed, prec, err, cfg["shape"], cfg["params"], cfg["bcs"])


def test_random_configurations_through_the_server():
    """The 2-D random configurations submitted together to the batched server (a few
    steps each): each result is bitwise the single-grid result of the same solve."""
    from paper_1909_13263_amd import workloads as W
    cfgs = [c for c in (RC.random_config(s) for s in range(40)) if len(c["shape"]) == 2]
    probs = []
    for k, c in enumerate(cfgs):
        probs.append((W.Problem(f"random{k}", c["shape"], c["lo"], c["hi"], c["bcs"], c["ham"],
                                c["params"], 0.01), c))
    srv = hjw.Server(hjw.FP32_MIXED, pool_bytes=128 << 20, max_active=16)
    ids = {srv.submit(p, c["phi"], scheme=c["scheme"]): (p, c) for p, c in probs}
    results = {r.rid: r for r in srv.drain()}
    srv.close()
    assert len(results) == len(probs)
    for sid, (p, c) in ids.items():
        g = hjw.Grid(c["shape"], c["lo"], c["hi"], c["bcs"], hjw.FP32_MIXED)
        g.set_hamiltonian(c["ham"], c["params"])
        if c["scheme"]:
            g.set_scheme(c["scheme"])
        g.set_phi(c["phi"])
        info = g.step_to(p.t_final, p.cfl)
        ref = g.get_phi()
        g.close()
        res = results[sid]
        assert res.status == hjw.OK
        assert res.info.steps == info.steps
        assert np.array_equal(res.phi, ref), (p.name, c["shape"], c["ham"], c["bcs"])
