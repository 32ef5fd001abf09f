"""FP64 parity with the oracle at the configurations' own final times.

The full-size configurations run far past the smooth regime the paper's tables cover:
the nonconvex -cos equation of Example 3.4 (Table 4's equation) to t = 1.0, the
level-set motion with extrapolated boundaries to t = 0.2, and Example 3.3's Burgers
equation past its kink time (the regime of Example 3.9).  Each is solved whole on the GPU
through the C ABI and by the FP64 oracle on the host cores, at sizes the oracle finishes
in seconds (the level set and -cos also at 512^2; Burgers at its full 1024^2), and every
node is compared:
  FP64            max|phi_gpu - phi_oracle| <= 1e-12 max|phi_oracle|;
  FP32 stencil    the L-inf / L1 (grid mean, both relative to max|phi|) bounds stated
                  per case, about 3x the errors measured on MI355X;
  FP32 storage    likewise.
Kinks make the weights switch sharply between neighbouring nodes, so these are the cases
where rounding differences between two correct implementations could grow.  In every case
above the FP64 difference stays at rounding level (printed).  The level set at 512^2 is
the exception, checked by the last test: near t = 0.2 the solution's growing plateaus meet,
and there the oracle itself moves by more than 1e-12 when phi0 is perturbed by one ulp.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1909_13263_amd import hjw
from paper_1909_13263_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64, MIXED, FP32 = hjw.FP64, hjw.FP32_MIXED, hjw.FP32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    yield


def _oracle(pr):
    prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)
    return O.step_to(prob, pr.phi0(), pr.t_final, pr.cfl)


def _gpu_solve(pr, prec):
    g = hjw.grid_for(pr, prec)
    g.set_phi(pr.phi0())
    info = g.step_to(pr.t_final, pr.cfl)
    phi = g.get_phi()
    g.close()
    return phi, info


# (id, problem, {prec: (L-inf bound, L1 bound) relative to max|phi|}); FP64 is always 1e-12
CASES = [
    # measured on MI355X (rel L-inf / L1): stencil 3.8e-8 / 1.8e-8, storage 1.6e-6 / 3.1e-7
    ("negcos-256-t1", lambda: W.negcos2d(256, 1.0), {MIXED: (1.2e-7, 6e-8), FP32: (5e-6, 1e-6)}),
    # stencil 5.3e-8 / 2.5e-8
    ("negcos-512-t1", lambda: W.negcos2d(512, 1.0), {MIXED: (1.6e-7, 8e-8)}),
    # stencil 5.0e-8 / 3.7e-9, storage 2.1e-5 / 4.2e-7
    ("levelset-256-t0.2", lambda: W.levelset2d(256, 0.2),
     {MIXED: (1.5e-7, 1.2e-8), FP32: (6e-5, 1.3e-6)}),
    # stencil 3.6e-8 / 4.0e-9
    ("burgers-1024-t1.5/pi^2", lambda: W.burgers2d(1024, 1.5 / math.pi**2),
     {MIXED: (1.1e-7, 1.2e-8)}),
]


@pytest.mark.parametrize("name,make,bounds", CASES, ids=[c[0] for c in CASES])
def test_whole_solve_to_the_configuration_horizon(name, make, bounds):
    pr = make()
    print(f"{name}: oracle {pr.shape} to t={pr.t_final:.5f}", flush=True)
    ref, info = _oracle(pr)
    scale = float(np.abs(ref).max())
    got, ginfo = _gpu_solve(pr, FP64)
    err = float(np.abs(got - ref).max()) / scale
    print(f"{name}: steps {ginfo.steps}/{info.steps} FP64 rel L-inf {err:.3e}", flush=True)
    assert ginfo.t == pr.t_final == info.t
    assert ginfo.steps == info.steps
    assert err <= 1e-12
    for prec, (linf_max, l1_max) in bounds.items():
        phi, pinfo = _gpu_solve(pr, prec)
        e = np.abs(phi - ref) / scale
        linf, l1 = float(e.max()), float(e.mean())
        print(f"{name}: prec={prec} steps {pinfo.steps} rel L-inf {linf:.3e} L1 {l1:.3e}",
              flush=True)
        assert pinfo.t == pr.t_final
        assert abs(pinfo.steps - info.steps) <= 1
        assert linf <= linf_max and l1 <= l1_max


def test_levelset_512_to_t02_within_the_problems_own_rounding_sensitivity():
    """The level set at 512^2 to t = 0.2 (410 steps), advanced in chunks of 50 steps on the
    GPU (FP64) and by the oracle, and by the oracle once more from phi0 perturbed by one ulp
    (seeded signs).  Through step 300 (t ~ 0.146) the GPU stays within 1e-12 of the oracle.
    Over the last 110 steps the problem amplifies rounding: the nodes where the plateaus of
    two circles meet (phi = -r of one circle beside the other's plateau) are flat to
    rounding, and the oracle's own one-ulp spread grows past 1e-12 there.  The final
    difference is held to 20 times that spread, measured here on the same run."""
    pr = W.levelset2d(512, 0.2)
    prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)
    phi0 = pr.phi0()
    rng = np.random.default_rng(7)
    ref = phi0.copy()
    per = phi0 * (1.0 + rng.choice([-1.0, 1.0], size=phi0.shape) * 2.0**-52)
    g = hjw.grid_for(pr, FP64)
    g.set_phi(phi0)
    t = 0.0
    steps = 0
    oracle_steps = 0   # the oracle's step_to counts the steps of each call
    while t < pr.t_final:
        ref, info = O.step_to(prob, ref, pr.t_final, pr.cfl, t0=t, max_steps=50)
        per, pinfo = O.step_to(prob, per, pr.t_final, pr.cfl, t0=t, max_steps=50)
        gi = g.step_to(pr.t_final, pr.cfl, max_steps=50)
        steps += 50
        oracle_steps += info.steps
        # alpha comes from derivative ranges that agree to rounding, so the checkpoint times
        # may differ in the last bits; the final step lands on t_final exactly in every run
        assert abs(gi.t - info.t) <= 1e-13 and abs(pinfo.t - info.t) <= 1e-13
        t = info.t
        scale = float(np.abs(ref).max())
        err = float(np.abs(g.get_phi() - ref).max()) / scale
        spread = float(np.abs(per - ref).max()) / scale
        print(f"levelset 512^2 step {min(steps, gi.steps)} t={t:.4f}: GPU-oracle {err:.3e}, "
              f"oracle one-ulp spread {spread:.3e}", flush=True)
        if steps <= 300:
            assert err <= 1e-12
    assert gi.t == info.t == pr.t_final and gi.steps == oracle_steps == 410
    assert err <= 20.0 * spread
    g.close()
