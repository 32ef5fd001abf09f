"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars: FP64 path max|phi_gpu - phi_oracle| <= 1e-12 max|phi_oracle|; derivatives to
1e-13 of their largest magnitude.  The FP32 paths (FP32 stencil with FP64 phi, and
FP32 phi) are held to the error bounds stated in each test, measured against the same
FP64 oracle.  Every input is a seeded synthetic field shaped like the paper's tests.
"""
import math
import os

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
    assert os.path.dirname(hjw.LIB_PATH).endswith("paper_1909_13263_amd")
    yield


def _oracle_problem(pr):
    return O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _field(shape, seed):
    rng = np.random.default_rng(seed)
    return W.random_smooth_periodic(shape, seed=seed) + 0.05 * rng.normal(size=shape)


# --------------------------------------------------------------------------- derivatives
DERIV_SHAPES = [(8,), (37,), (160,), (1030,), (2500,), (8, 8), (33, 65), (40, 70), (96, 130),
                (100, 200), (135, 260), (256, 256)]
DERIV_TOL = {FP64: 1e-13, MIXED: 2e-6, FP32: 2e-5}


@pytest.mark.parametrize("shape", DERIV_SHAPES)
@pytest.mark.parametrize("bc", [hjw.BC_PERIODIC, hjw.BC_EXTRAP])
@pytest.mark.parametrize("prec", [FP64, MIXED, FP32])
def test_derivatives_match_oracle(shape, bc, prec):
    """Steps 1-4: phi_x^-+ (and phi_y^-+) elementwise, ragged tiles and both boundaries."""
    phi = _field(shape, seed=sum(shape) + bc)
    lo = [0.0] * len(shape)
    hi = [0.05 * n for n in shape[::-1]]
    g = hjw.Grid(shape, lo, hi, bc, prec)
    g.set_phi(phi)
    got = [t.cpu().numpy() for t in g.derivatives()]
    h = tuple((hi[a] - lo[a]) / shape[::-1][a] for a in range(len(shape)))
    ref = O.derivatives(O.Problem(shape, h, O.H_LINEAR, (1.0, 0.0), bc), phi)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= DERIV_TOL[prec] * np.abs(b).max()
    g.close()


def test_derivatives_on_kinked_data_fp64():
    """Data with kinks exercise the antiderivative branch of the cell lengths."""
    pr = W.levelset2d(200)
    phi = pr.phi0()
    g = hjw.grid_for(pr, FP64)
    g.set_phi(phi)
    got = [t.cpu().numpy() for t in g.derivatives()]
    ref = O.derivatives(_oracle_problem(pr), phi)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


# --------------------------------------------------------------------------- single steps
STEP_CASES = [
    lambda: W.burgers1d(160), lambda: W.advect1d(37), lambda: W.negcos1d(50),
    lambda: W.burgers2d(96, ny=70), lambda: W.negcos2d(65, ny=33),
    lambda: W.levelset2d(100, ny=72), lambda: W.burgers2d(256),
    lambda: W.levelset2d(260, ny=135),
]
STEP_TOL = {FP64: 1e-14, MIXED: 1e-7, FP32: 1e-6}


@pytest.mark.parametrize("case", range(len(STEP_CASES)))
@pytest.mark.parametrize("prec", [FP64, MIXED, FP32])
def test_one_rk3_step_matches_oracle(case, prec):
    """One TVD-RK3 step (Step 5) with the LF flux (eq. LF) and the global dissipation."""
    pr = STEP_CASES[case]()
    phi = pr.phi0()
    ref, info = O.rk3_step(_oracle_problem(pr), phi, 0.0, pr.t_final, 0.5)
    g = hjw.grid_for(pr, prec)
    g.set_phi(phi)
    gi = g.step_to(pr.t_final, 0.5, max_steps=1)
    assert gi.steps == 1
    assert gi.last_dt == pytest.approx(info.last_dt, rel=1e-12 if prec == FP64 else 1e-5)
    assert gi.alpha_x == pytest.approx(info.alpha_x, rel=1e-12 if prec == FP64 else 1e-5)
    assert _rel(g.get_phi(), ref) <= STEP_TOL[prec]


SPIKES_2D = [(0, 0), (1, 0), (5, 3), (17, 7), (31, 15), (32, 8), (47, 1), (63, 15), (64, 0),
             (100, 20), (127, 31), (70, 16), (90, 29), (15, 17), (3, 30), (120, 5)]
SPIKES_1D = [0, 1, 63, 64, 255, 256, 300, 511, 599]


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_range_fold_finds_the_extreme_anywhere(prec):
    """The dissipation alpha (eq. LF) is set by the derivative range over the whole grid.
    A spike at one node makes the derivatives there the extremes; placed at nodes handled
    by different lanes, rows of lanes, waves and tiles, alpha and dt must follow it."""
    rel = 1e-12 if prec == FP64 else 1e-5
    base = W.burgers2d(128, ny=32)
    for x, y in SPIKES_2D:
        phi = 0.01 * base.phi0()
        phi[y, x] += 0.5 + 0.01 * x - 0.003 * y
        ref, info = O.rk3_step(_oracle_problem(base), phi, 0.0, base.t_final, 0.5)
        g = hjw.grid_for(base, prec)
        g.set_phi(phi)
        gi = g.step_to(base.t_final, 0.5, max_steps=1)
        g.close()
        span = max(abs(r) for r in info.range)
        assert np.allclose(gi.range, info.range, rtol=0, atol=rel * span), (x, y)
        assert gi.alpha_x == pytest.approx(info.alpha_x, rel=rel), (x, y)
        assert gi.alpha_y == pytest.approx(info.alpha_y, rel=rel), (x, y)
        assert gi.last_dt == pytest.approx(info.last_dt, rel=rel), (x, y)
    base1 = W.burgers1d(600)
    for x in SPIKES_1D:
        phi = 0.01 * base1.phi0()
        phi[x] -= 0.4 + 0.001 * x
        ref, info = O.rk3_step(_oracle_problem(base1), phi, 0.0, base1.t_final, 0.5)
        g = hjw.grid_for(base1, prec)
        g.set_phi(phi)
        gi = g.step_to(base1.t_final, 0.5, max_steps=1)
        g.close()
        span = max(abs(r) for r in info.range[:2])
        assert np.allclose(gi.range[:2], info.range[:2], rtol=0, atol=rel * span), x
        assert gi.alpha_x == pytest.approx(info.alpha_x, rel=rel), x
        assert gi.last_dt == pytest.approx(info.last_dt, rel=rel), x


# --------------------------------------------------------------------------- whole solves
def test_burgers1d_n160_full_solve():
    """Example 3.6's equation, N = 160, CFL 0.5, to t = 0.5/pi^2, FP64: within 1e-12."""
    pr = W.burgers1d(160)
    ref, info = O.step_to(_oracle_problem(pr), pr.phi0(), pr.t_final, 0.5)
    g = hjw.grid_for(pr, FP64)
    g.set_phi(pr.phi0())
    gi = g.step_to(pr.t_final, 0.5)
    assert gi.steps == info.steps and gi.t == pr.t_final
    assert _rel(g.get_phi(), ref) <= 1e-12


@pytest.mark.parametrize("n,t_final", [(128, 0.5 / math.pi**2), (128, 1.5 / math.pi**2),
                                       (256, 0.5 / math.pi**2)])
def test_burgers2d_full_solve(n, t_final):
    """Example 3.3 to the smooth time and past the kink time; FP64 within 1e-12, the FP32
    stencil with FP64 phi within 2e-6 and FP32 phi within 2e-5 of the FP64 oracle."""
    pr = W.burgers2d(n, t_final)
    ref, info = O.step_to(_oracle_problem(pr), pr.phi0(), t_final, 0.5)
    for prec, tol in [(FP64, 1e-12), (MIXED, 2e-6), (FP32, 2e-5)]:
        g = hjw.grid_for(pr, prec)
        g.set_phi(pr.phi0())
        gi = g.step_to(t_final, 0.5)
        assert gi.t == t_final
        assert abs(gi.steps - info.steps) <= (0 if prec == FP64 else 1)
        err = _rel(g.get_phi(), ref)
        print(f"burgers2d n={n} t={t_final:.4f} prec={prec} rel={err:.3e}")
        assert err <= tol


def test_negcos2d_full_solve():
    """Example 3.4's equation to t = 0.5/pi^2 at 160 x 160."""
    pr = W.negcos2d(160, 0.5 / math.pi**2)
    ref, _ = O.step_to(_oracle_problem(pr), pr.phi0(), pr.t_final, 0.5)
    for prec, tol in [(FP64, 1e-12), (MIXED, 2e-6), (FP32, 2e-5)]:
        g = hjw.grid_for(pr, prec)
        g.set_phi(pr.phi0())
        g.step_to(pr.t_final, 0.5)
        err = _rel(g.get_phi(), ref)
        print(f"negcos2d prec={prec} rel={err:.3e}")
        assert err <= tol


# --------------------------------------------------------------------------- full sizes
@pytest.mark.parametrize("make,steps", [(lambda: W.burgers2d(1024), 3),
                                        (lambda: W.negcos2d(2048), 2)])
def test_full_size_steps_match_oracle(make, steps):
    """The benchmark's shapes (1024^2 Burgers, 2048^2 -cos) in the launch configuration the
    benchmark times: a few whole steps against the oracle, every node compared."""
    pr = make()
    phi = pr.phi0()
    ref, info = O.step_to(_oracle_problem(pr), phi, pr.t_final, 0.5, max_steps=steps)
    for prec, tol in [(FP64, 1e-12), (MIXED, 1e-6)]:
        g = hjw.grid_for(pr, prec)
        g.set_phi(phi)
        gi = g.step_to(pr.t_final, 0.5, max_steps=steps)
        assert gi.steps == steps
        err = _rel(g.get_phi(), ref)
        print(f"{pr.name} {pr.shape} prec={prec} steps={steps} rel={err:.3e}")
        assert err <= tol
        g.close()


def test_levelset_4096_fp32_step():
    """The 4096^2 level-set problem in FP32 storage: one step against the FP64 oracle."""
    pr = W.levelset2d(4096)
    phi = pr.phi0()
    ref, _ = O.rk3_step(_oracle_problem(pr), phi, 0.0, pr.t_final, 0.5)
    g = hjw.grid_for(pr, FP32)
    g.set_phi(phi)
    g.step_to(pr.t_final, 0.5, max_steps=1)
    got = g.get_phi()
    err = float(np.abs(got - ref).max())
    print(f"levelset 4096 fp32 one step abs err {err:.3e}")
    assert err <= 2e-6


# --------------------------------------------------------------------------- invariants
def test_graph_replays_match_eager_launches():
    """Whole steps replayed from a captured HIP graph give the eager result bit for bit,
    on every replay, with eager work and synchronisation in between."""
    pr = W.burgers2d(192, 1.0 / math.pi**2)
    eager = hjw.grid_for(pr, MIXED)
    eager.set_option(hjw.OPT_USE_GRAPH, 0)
    graph = hjw.grid_for(pr, MIXED)
    eager.set_phi(pr.phi0())
    graph.set_phi(pr.phi0())
    for k in range(1, 5):
        t = pr.t_final * k / 4
        ie = eager.step_to(t, 0.5)
        ig = graph.step_to(t, 0.5)
        assert ie.steps == ig.steps and ie.t == ig.t
        assert np.array_equal(eager.get_phi(), graph.get_phi())
        _ = eager.derivatives()


@pytest.mark.parametrize("prec", [MIXED, FP32])
@pytest.mark.parametrize("shape", [(100, 200), (256, 256), (135, 260)])
def test_segment_lengths_give_identical_results(prec, shape):
    """4-node and 8-node sweeps (HJW_OPT_SEGMENT) compute every node with the same
    arithmetic: whole steps agree bit for bit."""
    pr = W.levelset2d(shape[1], 0.01, ny=shape[0])
    out = []
    for seg in (4, 8):
        g = hjw.grid_for(pr, prec)
        g.set_option(hjw.OPT_SEGMENT, seg)
        g.set_phi(pr.phi0())
        info = g.step_to(pr.t_final, pr.cfl)
        out.append((info.steps, g.get_phi()))
        g.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_plan_launch_gives_identical_results(prec):
    """The step plan computed in every workgroup of the second stage or in a launch of its
    own (HJW_OPT_PLAN) is the same computation on the same slots: identical bits."""
    pr = W.negcos2d(300, 0.05, ny=230)
    out = []
    for mode in (1, 2):
        g = hjw.grid_for(pr, prec)
        g.set_option(hjw.OPT_PLAN, mode)
        g.set_phi(pr.phi0())
        info = g.step_to(pr.t_final, pr.cfl)
        out.append((info.steps, info.last_dt, g.get_phi()))
        g.close()
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])


def test_transpose_symmetry_on_gpu():
    """Dimension by dimension: a transposed problem gives the transposed result, bit for
    bit: the row and column sweeps run the same arithmetic, and the products of the
    symmetric sums (H, the LF term, the dissipation) are kept out of fused multiply-adds."""
    pr = W.burgers2d(128)
    phi = pr.phi0() + 0.01 * W.random_smooth_periodic(pr.shape, seed=9)
    out = []
    for p in (phi, np.ascontiguousarray(phi.T)):
        g = hjw.grid_for(pr, FP64)
        g.set_phi(p)
        g.step_to(0.02, 0.5)
        out.append(g.get_phi())
    assert np.array_equal(out[0], out[1].T)


def test_reflection_symmetry_on_gpu():
    """x -> -x with H(p) -> H(-p) reflects the solution."""
    pr = W.burgers1d(160)
    phi = pr.phi0() + 0.1 * np.sin(3 * math.pi * pr.coords(0))
    a = hjw.grid_for(pr, FP64)
    a.set_phi(phi)
    a.step_to(0.03, 0.5)
    b = hjw.Grid(pr.shape, pr.lo, pr.hi, pr.bc, FP64)
    b.set_hamiltonian(hjw.H_BURGERS, (-1.0, 0.0, 1.0))
    b.set_phi(np.roll(phi[::-1], 1))
    b.step_to(0.03, 0.5)
    assert np.allclose(np.roll(b.get_phi()[::-1], 1), a.get_phi(), rtol=0, atol=1e-13)


def test_step_to_contract():
    pr = W.burgers2d(64, 0.03)
    g = hjw.grid_for(pr, FP64)
    g.set_phi(pr.phi0())
    i1 = g.step_to(0.01, 0.5, max_steps=2)
    assert i1.steps == 2 and i1.t < 0.01
    i2 = g.step_to(0.01, 0.5)
    assert i2.t == 0.01
    i3 = g.step_to(0.01, 0.5)      # nothing left to do
    assert i3.steps == i2.steps
    i4 = g.step_to(pr.t_final, 0.5)
    assert i4.t == pr.t_final


def test_non_finite_input_fails_the_grid():
    pr = W.burgers2d(64)
    g = hjw.grid_for(pr, FP64)
    phi = pr.phi0()
    phi[3, 5] = np.nan
    with pytest.raises(hjw.HJWError) as e:
        g.set_phi(phi)
    assert e.value.code == hjw.ENONFINITE
    with pytest.raises(hjw.HJWError) as e:
        g.step_to(0.01, 0.5)
    assert e.value.code == hjw.ESTATE
    g.set_phi(pr.phi0())            # recovers
    g.step_to(0.001, 0.5)


def test_blowup_is_reported():
    """A CFL number far above the stability limit makes phi overflow; the step that
    produces a non-finite value is reported and the grid is failed."""
    pr = W.burgers2d(64, 50.0)
    g = hjw.grid_for(pr, FP64)
    g.set_phi(pr.phi0() * 1e3)
    with pytest.raises(hjw.HJWError) as e:
        g.step_to(pr.t_final, 40.0)
    assert e.value.code == hjw.ENONFINITE


def test_workspace_too_small_is_rejected():
    import torch
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(hjw.HJWError) as e:
        hjw.Grid((256, 256), (0, 0), (1, 1), 0, FP64, workspace=ws)
    assert e.value.code == hjw.ENOMEM


def test_time_kernels_contract():
    """hjw_time_kernels returns positive per-launch durations and leaves phi unset."""
    pr = W.burgers2d(256)
    g = hjw.grid_for(pr, MIXED)
    g.set_phi(pr.phi0())
    ms = g.time_kernels(reps=3)
    assert ms["plan"] == 0.0                # a 256^2 grid plans inside the second stage
    assert all(ms[k] > 0 for k in ("pre", "mid", "last")), ms
    with pytest.raises(hjw.HJWError) as e:
        g.step_to(0.01, 0.5)
    assert e.value.code == hjw.ESTATE
    g.set_phi(pr.phi0())
    g.step_to(0.001, 0.5)


@pytest.mark.parametrize("pr", [W.timed2d(200, 0.8, -0.6, 5.0, 0.9, 0.05, ny=135),
                                W.burgers2d(2048, 0.002)], ids=["timed", "plan_launch"])
def test_time_kernels_then_solve_is_bitwise_a_fresh_solve(pr):
    """Timing a grid's kernels (a hold kernel, then repeated launches of each stage) and
    setting phi again gives the same solve as a grid that was never timed; the family with
    kernels of its own and a grid that plans in its own launch included."""
    g = hjw.grid_for(pr, MIXED)
    g.set_phi(pr.phi0())
    ms = g.time_kernels(reps=3)
    assert all(ms[k] > 0 for k in ("pre", "mid", "last")), ms
    assert (ms["plan"] > 0) == (pr.cells > 2048 * 64 * 16), ms
    g.set_phi(pr.phi0())
    gi = g.step_to(pr.t_final, pr.cfl)
    got = g.get_phi()
    g.close()
    f = hjw.grid_for(pr, MIXED)
    f.set_phi(pr.phi0())
    fi = f.step_to(pr.t_final, pr.cfl)
    assert gi.steps == fi.steps
    assert np.array_equal(got, f.get_phi())
    f.close()


# --------------------------------------------------------------------------- WENO-JP
JP_SHAPES = [(37,), (1030,), (8, 8), (33, 65), (100, 200), (135, 260), (256, 256)]


@pytest.mark.parametrize("shape", JP_SHAPES)
@pytest.mark.parametrize("bc", [hjw.BC_PERIODIC, hjw.BC_EXTRAP])
@pytest.mark.parametrize("prec", [FP64, MIXED, FP32])
def test_jp_derivatives_match_oracle(shape, bc, prec):
    """The comparison scheme (WENO-JP indicators): derivatives against the oracle's WENO-JP."""
    phi = _field(shape, seed=sum(shape) + 11 * bc)
    lo = [0.0] * len(shape)
    hi = [0.05 * n for n in shape[::-1]]
    g = hjw.Grid(shape, lo, hi, bc, prec)
    g.set_scheme(hjw.WENO_JP)
    g.set_phi(phi)
    got = [t.cpu().numpy() for t in g.derivatives()]
    h = tuple((hi[a] - lo[a]) / shape[::-1][a] for a in range(len(shape)))
    ref = O.derivatives(O.Problem(shape, h, O.H_LINEAR, (1.0, 0.0), bc, scheme=O.WENO_JP), phi)
    for a, r in zip(got, ref):
        assert np.abs(a - r).max() <= DERIV_TOL[prec] * np.abs(r).max()


@pytest.mark.parametrize("make", [lambda: W.burgers2d(128, 1.5 / math.pi**2),
                                  lambda: W.negcos2d(160, 0.5 / math.pi**2),
                                  lambda: W.levelset2d(120, 0.05)])
def test_jp_whole_solves_match_oracle(make):
    """WENO-JP whole solves: FP64 within 1e-12 of the oracle, the FP32 stencil within 2e-6."""
    pr = make()
    ref, info = O.step_to(O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc,
                                    scheme=O.WENO_JP), pr.phi0(), pr.t_final, 0.5)
    for prec, tol in [(FP64, 1e-12), (MIXED, 2e-6)]:
        g = hjw.grid_for(pr, prec, scheme=hjw.WENO_JP)
        g.set_phi(pr.phi0())
        gi = g.step_to(pr.t_final, 0.5)
        assert abs(gi.steps - info.steps) <= (0 if prec == FP64 else 1)
        err = _rel(g.get_phi(), ref)
        print(f"JP {pr.name} {pr.shape} prec={prec} rel={err:.3e}")
        assert err <= tol


def test_jp_full_size_steps_match_oracle():
    """WENO-JP at the 1024^2 benchmark shape: three whole steps against the oracle."""
    pr = W.burgers2d(1024)
    ref, _ = O.step_to(O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc,
                                 scheme=O.WENO_JP), pr.phi0(), pr.t_final, 0.5, max_steps=3)
    for prec, tol in [(FP64, 1e-12), (MIXED, 1e-6)]:
        g = hjw.grid_for(pr, prec, scheme=hjw.WENO_JP)
        g.set_phi(pr.phi0())
        g.step_to(pr.t_final, 0.5, max_steps=3)
        assert _rel(g.get_phi(), ref) <= tol
        g.close()


def test_scheme_switch_applies_to_the_next_step():
    """hjw_set_scheme between steps: WENO-L then WENO-JP equals the oracle doing the same."""
    pr = W.burgers2d(96, 0.02)
    g = hjw.grid_for(pr, FP64)
    g.set_phi(pr.phi0())
    g.step_to(0.01, 0.5)
    g.set_scheme(hjw.WENO_JP)
    g.step_to(0.02, 0.5)
    prob_l = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)
    prob_j = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc, scheme=O.WENO_JP)
    ref, info = O.step_to(prob_l, pr.phi0(), 0.01, 0.5)
    t = info.t
    while t < 0.02:                          # continue from t = 0.01 with the other scheme
        ref, info = O.rk3_step(prob_j, ref, t, 0.02, 0.5)
        t = info.t
    assert _rel(g.get_phi(), ref) <= 1e-12
