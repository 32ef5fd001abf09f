"""FP32 error bounds of the full-size configurations, whole solves on the GPU.

Each configuration is solved to its final time in FP64 and in the FP32 path(s) it is
quoted with.  The FP64 GPU path matches the FP64 oracle to 1e-12 of max|phi| (whole
solves at reduced size and a few whole steps at these sizes in test_gpu_parity.py);
solving these sizes to the final time on the CPU oracle would take hours, so the FP64
GPU result stands in for it here.  L1 is the grid mean of |error|.

Bounds (about 2-4x the measured errors):
  Burgers 1024^2, t = 0.5/pi^2   stencil L-inf 1e-7,  L1 2e-8;  storage L-inf 5e-6, L1 1e-6
  Burgers 1024^2, t = 1.5/pi^2   stencil L-inf 2e-7,  L1 2e-8;  storage L-inf 2e-5, L1 3e-6
  -cos 2048^2,    t = 1.0        stencil L-inf 1.5e-7, L1 6e-8
  level set 4096^2, t = 0.2      stencil L-inf 1e-3,  L1 2e-6;  storage L-inf 1e-3, L1 1e-5
"""
import math

import numpy as np
import pytest

from paper_1909_13263_amd import hjw
from paper_1909_13263_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64, MIXED, FP32 = hjw.FP64, hjw.FP32_MIXED, hjw.FP32

CASES = [
    ("burgers-smooth", lambda: W.burgers2d(1024, 0.5 / math.pi**2),
     {MIXED: (1e-7, 2e-8), FP32: (5e-6, 1e-6)}),
    ("burgers-kinks", lambda: W.burgers2d(1024, 1.5 / math.pi**2),
     {MIXED: (2e-7, 2e-8), FP32: (2e-5, 3e-6)}),
    ("negcos-2048", lambda: W.negcos2d(2048, 1.0), {MIXED: (1.5e-7, 6e-8)}),
    ("levelset-4096", lambda: W.levelset2d(4096, 0.2), {MIXED: (1e-3, 2e-6), FP32: (1e-3, 1e-5)}),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    yield


def _solve(pr, prec):
    g = hjw.grid_for(pr, prec)
    g.set_phi(pr.phi0())
    info = g.step_to(pr.t_final, pr.cfl)
    phi = g.get_phi()
    g.close()
    assert info.t == pr.t_final
    return phi, info


@pytest.mark.parametrize("name,make,bounds", CASES, ids=[c[0] for c in CASES])
def test_fp32_error_bounds_at_full_size(name, make, bounds):
    pr = make()
    ref, info = _solve(pr, FP64)
    assert np.isfinite(ref).all()
    for prec, (linf_max, l1_max) in bounds.items():
        phi, pinfo = _solve(pr, prec)
        err = np.abs(phi - ref)
        linf, l1 = float(err.max()), float(err.mean())
        print(f"{name} prec={prec} steps={pinfo.steps}/{info.steps} linf={linf:.3e} l1={l1:.3e}")
        assert abs(pinfo.steps - info.steps) <= 1
        assert linf <= linf_max and l1 <= l1_max


def test_burgers_1024_fp64_whole_solve_matches_oracle():
    """The 1024^2 Burgers configuration solved to t = 0.5/pi^2 (215 steps) in FP64 on the
    GPU and by the FP64 oracle on the host cores: every node within 1e-12 of max|phi|."""
    import oracle as O
    pr = W.burgers2d(1024, 0.5 / math.pi**2)
    phi0 = pr.phi0()
    ref, info = O.step_to(O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc), phi0,
                          pr.t_final, pr.cfl)
    got, ginfo = _solve(pr, FP64)
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"burgers 1024^2 FP64 whole solve: steps {ginfo.steps}/{info.steps} rel {err:.3e}")
    assert ginfo.steps == info.steps
    assert err <= 1e-12


def test_grid_of_more_than_2_31_nodes_is_its_periodic_cell_tiled():
    """64-bit indexing at the size HBM allows: a periodic 49152 x 49152 grid (2.4e9 nodes,
    above 2^31; 68 GB of FP32-stencil workspace, plan in its own launch over 2.36 M tiles)
    holding data of period 1024 in both axes.  Every node sees the stencil values and the
    derivative box of the 1024 x 1024 grid, so two steps give that grid's result tiled
    48 x 48, bit for bit; the 1024 x 1024 result matches the oracle (test_gpu_parity.py)."""
    import torch
    p, reps = 1024, 48
    n = p * reps
    small = W.burgers2d(p, 1.0)
    g = hjw.grid_for(small, MIXED)
    g.set_phi(small.phi0())
    gi = g.step_to(small.t_final, small.cfl, max_steps=2)
    ref = torch.from_numpy(g.get_phi()).cuda()
    g.close()
    lo = small.lo
    hi = tuple(l + reps * (h - l) for l, h in zip(small.lo, small.hi))
    big = hjw.Grid((n, n), lo, hi, hjw.BC_PERIODIC, MIXED)
    big.set_hamiltonian(small.ham, small.params)
    phi = torch.from_numpy(small.phi0()).cuda().repeat(reps, reps)   # 19 GB, FP64
    big.set_phi(phi)
    bi = big.step_to(small.t_final, small.cfl, max_steps=2)
    big.get_phi_device(out=phi)
    big.close()
    assert bi.steps == gi.steps == 2
    assert bi.last_dt == gi.last_dt and bi.alpha_x == gi.alpha_x and bi.range == gi.range
    blocks = phi.view(reps, p, reps, p)
    for r in range(reps):
        assert torch.equal(blocks[r], ref[:, None, :].expand(p, reps, p)), r
    del phi, blocks
    torch.cuda.empty_cache()
